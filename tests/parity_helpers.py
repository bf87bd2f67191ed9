"""Shared parity bars of the GPU tests (imported by the test modules; no
tests here).  The oracle is the FP64 CPU decoder in oracle/."""
import os

import numpy as np

NT = min(16, os.cpu_count() or 1)


def fp32_decode_bar(agree, ref_lsd, gpu_lsd, min_q_gap, L, n_cols, min_abs_post):
    """The FP32 bar on whole decodes, per shot: agree (corrections equal),
    ref_lsd / gpu_lsd (LSD ran on the oracle / the GPU), min_q_gap and
    min_abs_post (the oracle's witnesses).  Shots a BP member decides (on
    either side) agree on >= 99.9%.  Every other disagreement sits at a tie:
    the shot reaches LSD on both sides and either
      * among the oracle's own LSD rank decisions (which column a cluster
        takes next, the order of a cluster's columns) one has a gap below
        1e-3 of the RMS scale of the normalised average, L / sqrt(n); FP32
        posteriors, which agree with FP64 to ~1e-6 relative, can order such
        a pair either way; or
      * some member of the oracle's decode took a decision with |L_v| below
        1e-3 (the message-level excuse): FP32 can take it the other way,
        that member then follows another trajectory, and its posterior is
        part of LSD's input.
    Over the shots that are at neither kind of tie, agreement is >= 99.9%.
    Returns the report line."""
    agree = np.asarray(agree, bool)
    min_q_gap = np.asarray(min_q_gap, np.float64)
    min_abs_post = np.asarray(min_abs_post, np.float64)
    bp_dec = ~np.asarray(ref_lsd, bool) | ~np.asarray(gpu_lsd, bool)
    dq = 1e-3 * L / np.sqrt(n_cols)
    rank_tie = min_q_gap < dq
    member_tie = min_abs_post < 1e-3
    tie = ~bp_dec & (rank_tie | member_tie)
    if bp_dec.any():
        assert agree[bp_dec].mean() >= 0.999, (agree[bp_dec].mean(), np.flatnonzero(bp_dec & ~agree)[:10])
    rest = ~agree & ~bp_dec
    assert tie[rest].all(), (np.flatnonzero(rest & ~tie)[:10], dq)
    firm = ~tie
    if firm.any():
        assert agree[firm].mean() >= 0.999, (agree[firm].mean(), np.flatnonzero(firm & ~agree)[:10])
    diff_rank = int((rest & rank_tie).sum())
    return (f"overall agreement {agree.mean():.5f} of {len(agree)} (target 0.999); "
            f"{agree[firm].mean() if firm.any() else 1.0:.5f} of the {int(firm.sum())} shots not at a tie; "
            f"{int(tie.sum())} shots at a tie (LSD rank gap < {dq:.3g}, or a member decision |L| < 1e-3), "
            f"{int((tie & ~agree).sum())} of them differ ({diff_rank} at a rank tie, "
            f"{int((rest & ~rank_tie).sum())} only at a member tie); "
            f"BP-decided {agree[bp_dec].mean() if bp_dec.any() else 1.0:.5f} of {int(bp_dec.sum())}")


def check_valid(dem, e, synd, st):
    """H e = s on every shot LSD did not flag, observables from e."""
    ok = (st[:, 0] & 4) == 0
    H = dem.dense_h().astype(np.int64)
    assert np.array_equal((e[ok].astype(np.int64) @ H.T) % 2, synd[ok])


def sampled_oracle_parity(dem, G, synd, e, st, n_sample, seed, label, schedule="serial", lsd_order=0):
    """Corrections of a sample of the shots of one request (decoded by the
    HIP path as e [B, n] with stats st) against the oracle run on the same
    shots with the graph's own schedules and settings, to the FP32 bar (or
    bit for bit for FP64 graphs).  Returns the report line."""
    from oracle import oracle as O

    B = synd.shape[0]
    if B == 0:
        return f"{label}: empty"
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(B, min(n_sample, B), replace=False))
    info = G.info()
    L, M, T = info["L"], info["M"], info["T_max"]
    ref = O.decode(O.OracleGraph(dem), G.schedules(), synd[pick], L=L, M=M, T=T, threads=NT,
                   schedule=schedule, lsd_order=lsd_order)
    agree = (ref["ehat"] == e[pick]).all(1)
    if info["message_bits"] == 64:
        assert agree.mean() >= 0.999, (label, agree.mean())
        return f"{label}: FP64 agreement {agree.mean():.5f} of {len(pick)} sampled shots"
    line = fp32_decode_bar(agree, ref["lsd_used"], (st[pick, 0] & 2) != 0, ref["min_q_gap"], L, dem.n,
                           ref["min_abs_post"])
    return f"{label}: {len(pick)} sampled shots: {line}"
