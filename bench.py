"""Benchmark of the batched VibeLSD decoder on one MI355X.

Workload: the 6.6.6 colour code at d = 9 over 9 rounds of a fixed-CNOT-order
X/Z syndrome-extraction circuit with uniform depolarising noise p = 1e-3,
as a detector error model from synth/ (m = 540 detectors, n = 16782
mechanisms, 70811 edges); L = 32 serial schedules, M = 5, T_max = 20,
alpha = 0.625, LSD-0.  Synthetic, seeded syndromes stand in for the paper's
circuits and data.

One step = vibe_decode over one batch of B shots (all of BP ensemble,
selection, LSD and observables), syndromes already resident in HBM.
Prints one JSON line.  Extra legs: serving (continuous batching of one-shot
requests from circuit-level codes d = 9, 13, 17 mixed 50/30/20 at p = 5e-4 and 1e-3, Poisson
arrivals at 0.5x and 0.8x the sustained rate, p50/p99 latency); a ragged
batch of circuit-level codes at d = 5..13 (rounds = d) decoded as one call
against one call per code;
the phenomenological workload (d = 11, 11 rounds, L = 32, T = 50) with
LSD-0 and with LSD order 10; the code-capacity workload (d = 5, 10^4 shots)
with its BP edge-update rate; fitting the channel LLRs and scaling factor
with the differentiable decoder (d = 5 circuit-level), fitted against
untuned decoder on held-out shots; the backward pass of the differentiable decoder (16 unrolled iterations of
the d = 5 circuit-level graph, 4096 shots, L = 32, FP32) with its own
roofline; the layered (check-serial) schedule on 8192 of the shots; BP+LSD-0
without ensembling (one member,
parallel schedule) on the same batch, with LSD calls and largest-cluster
sizes beside VibeLSD's (the comparison of the paper's Sec. IV.H); the
per-shot-launch form
(vibe_decode_plain, one launch sequence per shot) on the first shots of the
batch, latency of small batches (64 shots per call, wall clock from
submission to completion), the oracle on a bounded sample of the host cores,
and the dominant kernel's roofline from HIP events around its launches.
HBM traffic per launch comes from the committed rocprofv3 counter summary
when it was taken on the same kernel source and launch size, else null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# algorithmic HBM bytes of one edge-update of the serial sweep: the previous
# message of the edge is read (its sign) and the new one written, FP32 each
BYTES_PER_EDGE_UPDATE = 8.0


PROFILE = os.path.join(ROOT, "profiles", "bp_ensemble_kernel_circuit_d9_r9_p1e-3.txt")
KERNEL_SOURCES = ("bp.hip", "internal.h", "graph.hip")
GRAD_PROFILE = os.path.join(ROOT, "profiles", "bp_grad_kernel_circuit_d5_r5_p1e-3.txt")
GRAD_SOURCES = ("grad.hip", "internal.h", "graph.hip")


def measured_traffic(launch_shots, profile=PROFILE, sources=KERNEL_SOURCES, key="traffic_launch_shots"):
    """HBM bytes per launch of a kernel from its committed counter summary, if
    the counters were taken on the same kernel sources at the same launch
    size; else None."""
    try:
        lines = open(profile).read().splitlines()
    except OSError:
        return None
    src = "".join(open(os.path.join(ROOT, "paper_2508_15743_amd", "csrc", f)).read() for f in sources)
    sha = hashlib.sha256(src.encode()).hexdigest()[:16]
    vals = dict(l.split()[:2] for l in lines if l.startswith(("source_sha256_16 ", key + " ",
                                                                "traffic_bytes_per_launch ")))
    if vals.get("source_sha256_16") != sha or vals.get(key) != str(launch_shots):
        return None
    return float(vals["traffic_bytes_per_launch"])


def ragged_leg(P, torch, shots, seed, tune=True, per_call=20000):
    """Circuit-level codes d = 5, 7, 9, 11, 13 (rounds = d, p = 1e-3) in one
    ragged call against one vibe_decode per code on the same syndromes.
    With `tune`, each graph is first autotuned on up to 2048 of its shots
    (slab placement, shots per wavefront, decision placement, grid) and
    both paths run with the chosen settings; the choices are reported.
    More than `per_call` shots per code run as several calls of at most
    that many per code on both paths (20000 per code fit one round of the
    ragged planner: one persistent BP launch over the five codes)."""
    from synth.dem import circuit_dem
    from synth.sample import permutations, sample

    cfgs = [(5, 32, 5, 20), (7, 32, 5, 20), (9, 32, 5, 20), (11, 32, 5, 20), (13, 64, 7, 25)]
    pairs, tuned = [], []
    for d, L, M, T in cfgs:
        dem = circuit_dem(d, d, 1e-3)
        G = P.Graph.from_dem(dem, permutations(dem.n, L, seed + d), L=L, M=M, T_max=T, alpha=0.625)
        s = torch.from_numpy(sample(dem, shots, seed + 100 + d).syndromes).to("cuda:0")
        if tune:
            ch = G.autotune(s[:min(shots, 2048)])
            tuned.append({"code": f"circuit_d{d}_r{d}_p0.001", **{k: ch[k] for k in
                          ("shots_per_wave", "decisions_global", "grid", "slab_in_lds", "from_cache")},
                          "sample_ms": round(ch["ms"], 2)})
            log(f"autotune d={d}: {ch}")
        pairs.append((G, s))
    rt = P.Runtime()
    outs = [P.Runtime.outputs(G, s) for G, s in pairs]
    pieces = [(a, min(a + per_call, shots)) for a in range(0, shots, per_call)]
    warm = min(shots, 1024)  # kernels, schedules and workspace of the small call
    rt.decode([(G, s[:warm]) for G, s in pairs])
    torch.cuda.synchronize()
    log(f"ragged mix: {shots} shots per code, {len(pieces)} ragged call(s)")
    t0 = time.perf_counter()
    for a, b in pieces:
        rt.decode([(G, s[a:b]) for G, s in pairs], outs=[tuple(x[a:b] for x in o) for o in outs])
        torch.cuda.synchronize()
        if len(pieces) > 1:
            log(f"  ragged call over shots {a}..{b} of each code done at {time.perf_counter() - t0:.1f}s")
    t_ragged = time.perf_counter() - t0
    log(f"ragged mix: {shots} shots per code, {len(pieces)} call(s) per code")
    t_code = []
    for (G, s), o in zip(pairs, outs):
        t0 = time.perf_counter()
        for a, b in pieces:
            G.decode(s[a:b], out=tuple(x[a:b] for x in o))
            if len(pieces) > 1:
                torch.cuda.synchronize()
                log(f"  call over shots {a}..{b} of one code done at {time.perf_counter() - t0:.1f}s")
        torch.cuda.synchronize()
        t_code.append(time.perf_counter() - t0)
    t_sep = sum(t_code)
    total = shots * len(cfgs)
    res = {"codes": [f"circuit_d{d}_r{d}_p0.001" for d, *_ in cfgs], "shots_per_code": shots,
           "calls_per_code": len(pieces),
           "ragged_shots_per_s": round(total / t_ragged, 1), "separate_shots_per_s": round(total / t_sep, 1),
           "ragged_over_separate": round(t_sep / t_ragged, 3),
           "separate_s_per_code": [round(t, 3) for t in t_code], "autotuned": tuned if tune else None}
    log(f"ragged mix d=5..13: {total / t_ragged:.0f} shots/s in one call, {total / t_sep:.0f} in one call per code")
    rt.close()
    for G, _ in pairs:
        G.close()
    return res


# algorithmic HBM bytes of one edge-iteration of the adjoint: the forward
# sweep reads the old message and writes the new one (8 B); the reverse
# sweep reads the checkpointed message and reads and writes its adjoint
# (12 B); FP32 each
GRAD_BYTES_PER_EDGE_ITER = 20.0


def phenom_leg(P, torch, seed, shots):
    """The phenomenological workload as configured (colour code d = 11, 11
    noisy rounds and a perfect one, p = q = 0.01; L = 32, M = 5, T = 50,
    FP32): LSD-0 against LSD order 10 on the same seeded shots, each graph
    autotuned first on 4096 of them."""
    from synth.dem import phenomenological_dem
    from synth.sample import permutations, sample

    dem = phenomenological_dem(11, 11, 0.01, 0.01)
    perms = permutations(dem.n, 32, seed + 5)
    b = sample(dem, shots, seed + 6)
    synd = torch.from_numpy(b.syndromes).to("cuda:0")
    out = {"workload": dem.name, "m": dem.m, "n": dem.n, "shots": shots}
    corr = {}
    for order in (0, 10):
        G = P.Graph.from_dem(dem, perms, L=32, M=5, T_max=50, lsd_order=order)
        G.decode(synd[:256])
        ch = G.autotune(synd[:min(shots, 4096)])
        torch.cuda.synchronize()
        P.vibe_profile_enable(G.handle, True)
        P.vibe_profile_read(G.handle)
        t1 = time.perf_counter()
        c, obs, st = G.decode(synd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        prof = P.vibe_profile_read(G.handle)
        G.close()
        st = st.cpu().numpy()
        corr[order] = c.cpu().numpy()
        out[f"lsd{order}"] = {"shots_per_s": round(shots / dt, 1),
                              "lsd_fraction": round(float(((st[:, 0] & 2) != 0).mean()), 5),
                              "lsd_kernel_ms": round(prof["lsd"][0], 3),
                              "bp_kernel_ms": round(prof["bp_ensemble"][0], 3),
                              "edge_updates_per_s": float(st[:, 7].astype(np.int64).sum()) * dem.nnz
                              / max(prof["bp_ensemble"][0] / 1e3, 1e-9),
                              "logical_error_rate": float((obs.cpu().numpy() != b.observables).any(1).mean()),
                              "autotune": {k: ch[k] for k in ("slab_in_lds", "grid", "shots_per_wave",
                                                               "decisions_global", "from_cache")}}
        log(f"phenomenological LSD-{order}: {shots / dt:.0f} shots/s, LSD kernel {prof['lsd'][0]:.1f} ms "
            f"(autotuned: {ch})")
    out["corrections_changed_by_order10"] = int((corr[0] != corr[10]).any(1).sum())
    return out


def code_capacity_leg(P, torch, seed, shots=10000):
    """The code-capacity workload as configured (colour code d = 5, p = 0.05,
    10^4 shots; L = 16, M = 5, T = 32, FP32), autotuned first on 4096 of its
    shots.  Its message slab fits in LDS, so the bound is LDS and issue, not
    HBM: edge-updates/s and the slab bytes they move (16 B per edge-update)
    are reported."""
    from synth.dem import code_capacity_dem
    from synth.sample import permutations, sample

    dem = code_capacity_dem(5, 0.05)
    b = sample(dem, shots, seed + 11)
    synd = torch.from_numpy(b.syndromes).to("cuda:0")
    G = P.Graph.from_dem(dem, permutations(dem.n, 16, seed + 10), L=16, M=5, T_max=32)
    G.decode(synd[:256])
    ch = G.autotune(synd[:min(shots, 4096)])
    torch.cuda.synchronize()
    P.vibe_profile_enable(G.handle, True)
    P.vibe_profile_read(G.handle)
    t1 = time.perf_counter()
    _, obs, st = G.decode(synd)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    prof = P.vibe_profile_read(G.handle)
    G.close()
    st = st.cpu().numpy()
    eu = float(st[:, 7].astype(np.int64).sum()) * dem.nnz / max(prof["bp_ensemble"][0] / 1e3, 1e-9)
    out = {"workload": dem.name, "m": dem.m, "n": dem.n, "nnz": dem.nnz, "shots": shots,
           "shots_per_s": round(shots / dt, 1), "bp_kernel_ms": round(prof["bp_ensemble"][0], 3),
           "edge_updates_per_s": eu, "lds_slab_bytes_per_s": 16.0 * eu,
           "lsd_fraction": round(float(((st[:, 0] & 2) != 0).mean()), 5),
           "logical_error_rate": float((obs.cpu().numpy() != b.observables).any(1).mean()),
           "autotune": {k: ch[k] for k in ("slab_in_lds", "grid", "shots_per_wave", "decisions_global",
                                            "from_cache")}}
    log(f"code capacity: {shots / dt:.0f} shots/s, {eu:.3g} edge-updates/s (autotuned: {ch})")
    return out


def tuning_leg(P, torch, seed, steps=30):
    """Fit the channel LLRs and one shared scaling factor with the
    differentiable decoder (K = 8 unrolled iterations, 8 members, 2048
    training shots of the d = 5 circuit-level graph, 30 Adam steps), then
    decode 32768 held-out shots with the untuned decoder (priors,
    alpha = 0.625) and the fitted one, both with L = 32, M = 5, T = 20."""
    from paper_2508_15743_amd import tune
    from synth.dem import circuit_dem
    from synth.sample import permutations, sample

    dem = circuit_dem(5, 5, 1e-3)
    perms = permutations(dem.n, 32, seed + 7)
    lam0 = np.log((1 - dem.priors) / dem.priors)
    K = 8
    train = torch.from_numpy(sample(dem, 2048, seed + 8).syndromes).to("cuda:0")
    held = sample(dem, 32768, seed + 9)
    held_s = torch.from_numpy(held.syndromes).to("cuda:0")
    Gt = P.Graph.from_dem(dem, perms[:8], L=8, M=1, T_max=K)
    t1 = time.perf_counter()
    lam, alpha, losses = tune.fit(Gt, train, K, steps=steps, lam0=lam0)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t1

    def heldout_loss(l, a):
        return float(Gt.bp_grad(held_s[:2048], torch.tensor(l), torch.full((K,), a))[0].item()) / 2048

    out = {"workload": dem.name, "train_shots": 2048, "members": 8, "K": K, "steps": steps,
           "fit_seconds": round(fit_s, 2), "loss_train_first_best": [round(losses[0], 5), round(min(losses), 5)],
           "loss_heldout": {"untuned": round(heldout_loss(lam0, 0.625), 5),
                            "tuned": round(heldout_loss(lam, alpha), 5)},
           "alpha_tuned": round(alpha, 5), "lambda_change_rms": round(float(np.sqrt(np.mean((lam - lam0) ** 2))), 5)}
    Gt.close()
    for name, pri, a in (("untuned", dem.priors, 0.625), ("tuned", tune.priors_from_llr(lam), alpha)):
        G = P.Graph(dem.h_indptr, dem.h_indices, pri, dem.l_indptr, dem.l_indices, perms, m=dem.m, n=dem.n,
                    L=32, M=5, T_max=20, alpha=a)
        G.decode(held_s[:256])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, obs, st = G.decode(held_s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        st = st.cpu().numpy()
        out[name] = {"shots_per_s": round(held.syndromes.shape[0] / dt, 1),
                     "logical_error_rate": float((obs.cpu().numpy() != held.observables).any(1).mean()),
                     "lsd_fraction": round(float(((st[:, 0] & 2) != 0).mean()), 5),
                     "member_iterations_per_shot": round(float(st[:, 7].mean()), 2)}
        G.close()
    log(f"tuning: loss/shot {losses[0]:.4f} -> {min(losses):.4f} (held-out {out['loss_heldout']['untuned']} -> "
        f"{out['loss_heldout']['tuned']}), LER {out['untuned']['logical_error_rate']:.2e} -> "
        f"{out['tuned']['logical_error_rate']:.2e}, LSD {out['untuned']['lsd_fraction']} -> {out['tuned']['lsd_fraction']}")
    return out


def grad_leg(P, torch, seed, batch, K):
    """Backward pass through K unrolled iterations (the differentiable
    decoder): d = 5 circuit-level graph (rounds 5, p = 1e-3), L = 32 serial
    members, FP32 messages, alpha_t = 0.625 and lambda from the priors;
    loss and gradients of a batch of syndromes, timed with HIP events on the
    stream of the launch."""
    from synth.dem import circuit_dem
    from synth.sample import permutations, sample

    dem = circuit_dem(5, 5, 1e-3)
    L = 32
    G = P.Graph.from_dem(dem, permutations(dem.n, L, seed + 5), L=L, M=5, T_max=20, alpha=0.625)
    s = torch.from_numpy(sample(dem, batch, seed + 6).syndromes).to("cuda:0")
    pri = np.asarray(dem.priors, dtype=np.float64)
    lam = torch.tensor(np.log((1.0 - pri) / pri), dtype=torch.float32, device="cuda:0")
    alpha = torch.full((K,), 0.625, dtype=torch.float32, device="cuda:0")
    G.bp_grad(s, lam, alpha)  # warm-up (workspace)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    loss, dlam, dalpha = G.bp_grad(s, lam, alpha)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    edge_iters = batch * L * K * dem.nnz
    achieved = GRAD_BYTES_PER_EDGE_ITER * edge_iters / sec / 1e9
    res = {"workload": "colour666_d5_r5_circuit_uniform_p0.001", "n": dem.n, "m": dem.m, "nnz": dem.nnz,
           "batch": batch, "L": L, "K": K, "dtype": "f32", "ms": round(1e3 * sec, 3),
           "shots_per_s": round(batch / sec, 1), "edge_iterations_per_s": edge_iters / sec,
           "loss": float(loss.item()), "grad_finite": bool(torch.isfinite(dlam).all() and torch.isfinite(dalpha).all()),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(batch, GRAD_PROFILE, GRAD_SOURCES, "traffic_launch_batch"),
                        "kernel": "bp_grad_kernel"}}
    log(f"grad: {batch} shots x {L} members x K={K} in {1e3 * sec:.1f} ms = {batch / sec:.0f} shots/s, "
        f"{achieved:.0f} GB/s algorithmic")
    G.close()
    return res


def serving_leg(P, torch, seed, seconds, slots=4):
    """One-shot requests (one window of d rounds each) from circuit-level codes
    d = 9, 13, 17 mixed 50/30/20, each at p = 5e-4 or 1e-3 with equal odds
    (six resident graphs; L/M/T = 32/5/20 at d = 9, 64/7/25 above), through
    the continuous-batching server (one graph per batch, each batch admitted
    by its HBM footprint from the server's pool): the single-shot latency
    of each code alone, the sustained rate of a burst, then Poisson arrivals
    at 0.5x and 0.8x that rate with p50/p99 latency from submission to
    completion, overall and per code."""
    import threading

    from synth.dem import circuit_dem
    from synth.sample import permutations, sample

    cfgs = [(d, p, L, M, T, w / 2) for d, L, M, T, w in ((9, 32, 5, 20, 0.5), (13, 64, 7, 25, 0.3),
                                                         (17, 64, 7, 25, 0.2)) for p in (5e-4, 1e-3)]
    rng = np.random.default_rng(seed)
    graphs, pools = [], []
    for d, p, L, M, T, _ in cfgs:
        dem = circuit_dem(d, d, p)
        graphs.append(P.Graph.from_dem(dem, permutations(dem.n, L, seed + d), L=L, M=M, T_max=T, alpha=0.625))
        pools.append(torch.from_numpy(sample(dem, 4096, seed + 300 + d + int(p * 1e4)).syndromes).to("cuda:0"))
    torch.cuda.synchronize()
    dists = sorted({c[0] for c in cfgs})
    # single-shot latency of each code alone (p = 1e-3 graphs, one shot per call)
    alone = {}
    for gi, (d, p, *_rest) in enumerate(cfgs):
        if p != 1e-3:
            continue
        G = graphs[gi]
        G.decode(pools[gi][:1])
        torch.cuda.synchronize()
        ts = []
        for i in range(12):
            t1 = time.perf_counter()
            G.decode(pools[gi][i + 1:i + 2])
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t1))
        alone[d] = round(float(np.median(ts)), 3)
    weights = np.array([c[5] for c in cfgs])
    srv = P.Server(graphs, slots=slots, max_batch_requests=512, max_batch_shots=1024)

    def run(n, rate):
        which = rng.choice(len(cfgs), size=n, p=weights / weights.sum())
        gaps = rng.exponential(1.0 / rate, size=n) if rate else np.zeros(n)
        tickets = [None] * n
        t0 = time.perf_counter()

        def producer():
            t_next = time.perf_counter()
            for i in range(n):
                t_next += gaps[i]
                while rate and time.perf_counter() < t_next:
                    pass
                g = int(which[i])
                tickets[i] = srv.submit(g, pools[g][i % 4096:i % 4096 + 1])[0]

        th = threading.Thread(target=producer)
        th.start()
        lat = []
        for i in range(n):
            while tickets[i] is None:
                time.sleep(1e-5)
            lat.append(srv.wait(tickets[i]))
        th.join()
        code = np.array([cfgs[int(w)][0] for w in which])
        return n / (time.perf_counter() - t0), np.array(lat), code

    run(256, 0)  # warm-up
    sustained, _, _ = run(3000, 0)
    res = {"codes": [f"circuit_d{d}_r{d}_p{p:g}" for d, p, *_ in cfgs], "mix": [c[5] for c in cfgs],
           "request": "one shot", "slots": slots, "sustained_requests_per_s": round(sustained, 1),
           "single_shot_ms_alone": {f"d{d}": alone[d] for d in dists}, "loads": []}
    for rho in (0.5, 0.8):
        rate = rho * sustained
        n = max(200, int(rate * seconds))
        got, lat, code = run(n, rate)
        per = {}
        for d in dists:
            sel = lat[code == d]
            if sel.size:
                per[f"d{d}"] = {"requests": int(sel.size), "p50_ms": round(float(np.percentile(sel, 50)), 3),
                                "p99_ms": round(float(np.percentile(sel, 99)), 3),
                                "p50_over_alone": round(float(np.percentile(sel, 50)) / alone[d], 2)}
        res["loads"].append({"offered": rho, "offered_requests_per_s": round(rate, 1),
                             "achieved_requests_per_s": round(got, 1),
                             "p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3), "per_code": per})
        log(f"serving at {rho:.1f}x of {sustained:.0f} req/s: p50 {np.percentile(lat, 50):.2f} ms, "
            f"p99 {np.percentile(lat, 99):.2f} ms; " +
            ", ".join(f"{k} p50 {v['p50_ms']:.1f} ms ({v['p50_over_alone']}x alone)" for k, v in per.items()))
    res.update(srv.info())
    srv.close()
    for G in graphs:
        G.close()
    return res


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1 << 15)
    ap.add_argument("--distance", type=int, default=9,
                    help="circuit-level code distance of the timed workload (profiling runs; 9 is the metric's)")
    ap.add_argument("--decisions-global", type=int, default=-1, choices=(-1, 0, 1),
                    help="with --no-autotune: K1 decision placement (-1 automatic)")
    ap.add_argument("--plain-shots", type=int, default=64)
    ap.add_argument("--latency-batches", type=int, default=200)
    ap.add_argument("--latency-batch", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-phenom", action="store_true", help="skip the phenomenological LSD-0 / LSD-10 leg")
    ap.add_argument("--no-tune", action="store_true", help="skip the parameter-fitting leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the headline graph with the default launch settings (profiling runs)")
    ap.add_argument("--phenom-shots", type=int, default=16384)
    ap.add_argument("--grad-batch", type=int, default=4096)
    ap.add_argument("--grad-K", type=int, default=16)
    ap.add_argument("--grad-only", action="store_true", help="run only the gradient leg (for profiling)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--ragged-only", action="store_true", help="run only the ragged leg")
    ap.add_argument("--serving-seconds", type=float, default=3.0, help="length of each offered-load run")
    ap.add_argument("--ragged-shots", type=str, default="128,1024", help="shots per code in the ragged leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--seed", type=int, default=2025)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the decoder shards by shots with no exchange, "
              "so the figure it reports is one GPU's throughput.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2508_15743_amd as P
    from synth.dem import circuit_dem
    from synth.sample import permutations, sample

    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 3 copies of 1 GiB")
        return

    if args.grad_only:
        print(json.dumps({"grad": grad_leg(P, torch, args.seed, args.grad_batch, args.grad_K)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_leg(P, torch, args.seed, args.serving_seconds)}), flush=True)
        return
    if args.ragged_only:
        print(json.dumps({"ragged": [ragged_leg(P, torch, int(k), args.seed) for k in args.ragged_shots.split(",")]}),
              flush=True)
        return

    # measured HBM ceiling: a 1 GiB device-to-device copy (read + write),
    # timed with events on the copy's stream
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write) against the {HBM_PEAK_GBS:.0f} GB/s specification")

    d, rounds, p = args.distance, args.distance, 1e-3
    L, M, T, alpha = (32, 5, 20, 0.625) if d <= 11 else (64, 7, 25, 0.625)
    t0 = time.time()
    dem = circuit_dem(d, rounds, p)
    perms = permutations(dem.n, L, args.seed)
    batch = sample(dem, args.batch, args.seed + 1)
    log(f"workload {dem.name}: m={dem.m} n={dem.n} nnz={dem.nnz}; sampled {args.batch} shots "
        f"in {time.time() - t0:.1f}s")
    G = P.Graph.from_dem(dem, perms, L=L, M=M, T_max=T, alpha=alpha)
    info = G.info()
    # the ceiling of the BP kernel's own access pattern: every resident
    # wavefront (24 per CU) streams a slab of this graph's size up and down,
    # reading and rewriting one 256-byte run per step (vibe_measure_slab_stream)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    waves, region = 24 * cus, 256 * max(int(info["chunks_max"]), 1)
    sbuf = torch.zeros(waves * region // 4, dtype=torch.float32, device=dev)
    st_ = torch.cuda.current_stream()
    P._check(P.lib().vibe_measure_slab_stream(P._ptr(sbuf), region, waves, 2, P._stream(st_)))
    e0.record(st_)
    P._check(P.lib().vibe_measure_slab_stream(P._ptr(sbuf), region, waves, 4, P._stream(st_)))
    e1.record(st_)
    torch.cuda.synchronize()
    stream_gbs = 2 * waves * region * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del sbuf
    log(f"slab stream ceiling: {stream_gbs:.0f} GB/s ({waves} wavefronts x {region} B)")
    synd = torch.from_numpy(batch.syndromes).to(dev)
    B = synd.shape[0]
    words = (dem.n + 63) // 64
    corr = torch.empty((B, words), dtype=torch.int64, device=dev)
    obs = torch.empty((B, 1), dtype=torch.uint8, device=dev)
    st = torch.empty((B, 8), dtype=torch.int32, device=dev)
    out = (corr, obs, st)
    # launch settings: timed on a sample of the batch, kept in the handle
    if args.no_autotune:
        G.set_launch(decisions_global=args.decisions_global)
        tune = {**G.get_launch(), "from_cache": False}
    else:
        tune = G.autotune(synd[:min(B, 4096)])
        log(f"autotune on {min(B, 4096)} shots: {tune}")

    for i in range(args.warmup):
        G.decode(synd, out=out)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    P.vibe_profile_enable(G.handle, True)
    P.vibe_profile_read(G.handle)  # clear
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    member_iters = 0
    for i in range(args.steps):
        G.decode(synd, out=out)
        torch.cuda.synchronize()
        member_iters += int(st[:, 7].sum().item())
        log(f"step {i + 1}/{args.steps} done at {time.perf_counter() - t_start:.2f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = P.vibe_profile_read(G.handle)
    P.vibe_profile_enable(G.handle, False)
    shots_per_s = B * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    stats = st.cpu().numpy()
    flags = stats[:, 0]
    lsd_frac = float(((flags & 2) != 0).mean())
    ler = float((obs.cpu().numpy() != batch.observables).any(1).mean())

    # dominant kernel: the BP ensemble; algorithmic bytes = edge-updates x 8 B
    bp_ms, bp_launches = prof["bp_ensemble"]
    edge_updates = member_iters * dem.nnz
    bp_s = bp_ms / 1e3
    achieved = BYTES_PER_EDGE_UPDATE * edge_updates / bp_s / 1e9 if bp_s > 0 else 0.0
    launch_shots = max(1, B // max(1, bp_launches // args.steps))
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "measured_peak": round(copy_gbs, 1), "frac_of_measured": round(achieved / copy_gbs, 4),
                # the committed counters were taken with the default settings:
                # one shot per wavefront, decisions in LDS
                "traffic": (measured_traffic(launch_shots)
                            if tune["shots_per_wave"] == 1 and tune["decisions_global"] != 1 else None),
                "slab_stream_ceiling": round(stream_gbs, 1),
                "kernel": "bp_ensemble_kernel",
                "avg_launch_ms": round(bp_ms / max(bp_launches, 1), 3),
                "edge_updates_per_s": edge_updates / bp_s if bp_s > 0 else 0.0,
                "kernel_ms": {k: round(v[0], 2) for k, v in prof.items()}}

    if roofline["traffic"]:
        moved = roofline["traffic"] / (bp_ms / max(bp_launches, 1) / 1e3) / 1e9
        roofline["moved_gbs"] = round(moved, 1)
        roofline["moved_frac_of_slab_stream_ceiling"] = round(moved / stream_gbs, 4)
    result = {
        "metric": "decoded shots/s at d=9 circuit-level p=1e-3, batched vs plain; p99 latency",
        "value": round(shots_per_s, 1),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded colour-code circuit-level DEM samples)",
        "config": {"workload": f"colour666_d{d}_r{rounds}_circuit_uniform_p{p:g}", "batch": B,
                   "m": dem.m, "n": dem.n, "nnz": dem.nnz, "L": L, "M": M, "T_max": T,
                   "alpha": alpha, "lsd_order": 0, "levels": [info["levels_min"], info["levels_max"]]},
        "roofline": roofline,
        "autotune": {k: tune[k] for k in ("slab_in_lds", "grid", "shots_per_wave", "decisions_global",
                                          "from_cache")},
        "lsd_fraction": round(lsd_frac, 5),
        "logical_error_rate": ler,
        "mean_member_iterations_per_shot": member_iters / (B * args.steps),
    }

    def cluster_stats(stats_np):
        lsd = (stats_np[:, 0] & 2) != 0
        big = stats_np[lsd, 5]
        pct = (lambda q: float(np.percentile(big, q)) if big.size else 0.0)
        return {"lsd_calls_per_5000": round(5000.0 * float(lsd.mean()), 1),
                "largest_cluster_p50": pct(50), "largest_cluster_p95": pct(95),
                "largest_cluster_max": int(big.max()) if big.size else 0}

    def baseline(dem_b, perms_b, synd_b, obs_b):
        """BP+LSD-0 without ensembling: one member, parallel schedule."""
        Gb = P.Graph.from_dem(dem_b, perms_b[:1], L=1, M=1, T_max=T, alpha=alpha, schedule="parallel")
        Gb.decode(synd_b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, bobs, bst = Gb.decode(synd_b)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        bler = float((bobs.cpu().numpy() != obs_b).any(1).mean())
        Gb.close()
        return dict(cluster_stats(bst.cpu().numpy()), shots_per_s=round(synd_b.shape[0] / dt, 1),
                    logical_error_rate=bler)

    comparison = {"vibelsd": cluster_stats(stats)}
    if not args.no_baseline:
        comparison["bp_lsd0"] = baseline(dem, perms, synd, batch.observables)
        log(f"BP+LSD-0 baseline: {comparison['bp_lsd0']['shots_per_s']:.0f} shots/s, LSD calls per 5000 "
            f"{comparison['bp_lsd0']['lsd_calls_per_5000']} vs VibeLSD {comparison['vibelsd']['lsd_calls_per_5000']}")
        # the same comparison under the Si1000 rates (the paper's Sec. IV.H
        # setting uses them), on 8192 shots
        dem_s = circuit_dem(d, rounds, p, noise="si1000")
        perms_s = permutations(dem_s.n, L, args.seed + 2)
        bs = sample(dem_s, 8192, args.seed + 3)
        synd_s = torch.from_numpy(bs.syndromes).to(dev)
        Gs = P.Graph.from_dem(dem_s, perms_s, L=L, M=M, T_max=T, alpha=alpha)
        _, sobs, sst = Gs.decode(synd_s)
        torch.cuda.synchronize()
        Gs.close()
        comparison["si1000"] = {"workload": dem_s.name, "shots": 8192,
                                "vibelsd": dict(cluster_stats(sst.cpu().numpy()),
                                                logical_error_rate=float((sobs.cpu().numpy() != bs.observables)
                                                                         .any(1).mean())),
                                "bp_lsd0": baseline(dem_s, perms_s, synd_s, bs.observables)}
        log(f"Si1000: LSD calls per 5000 {comparison['si1000']['bp_lsd0']['lsd_calls_per_5000']} (BP+LSD-0) "
            f"vs {comparison['si1000']['vibelsd']['lsd_calls_per_5000']} (VibeLSD)")
        # the layered (check-serial) schedule: the same ensemble size and
        # limits, members ordering the checks instead of the columns
        nl = min(B, 8192)
        Gl = P.Graph.from_dem(dem, permutations(dem.m, L, args.seed + 4), L=L, M=M, T_max=T, alpha=alpha,
                              schedule="layered")
        Gl.decode(synd[:256])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, lobs, lst = Gl.decode(synd[:nl])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        lst = lst.cpu().numpy()
        comparison["layered"] = dict(cluster_stats(lst), shots=nl, shots_per_s=round(nl / dt, 1),
                                     logical_error_rate=float((lobs.cpu().numpy() != batch.observables[:nl])
                                                              .any(1).mean()),
                                     mean_member_iterations_per_shot=float(lst[:, 7].mean()))
        Gl.close()
        log(f"layered schedule: {nl / dt:.0f} shots/s, LSD calls per 5000 "
            f"{comparison['layered']['lsd_calls_per_5000']}")
    result["comparison"] = comparison

    if not args.no_ragged:
        result["ragged"] = [ragged_leg(P, torch, int(k), args.seed) for k in args.ragged_shots.split(",")]
    if not args.no_serving:
        result["serving"] = serving_leg(P, torch, args.seed, args.serving_seconds)
    if not args.no_grad:
        result["grad"] = grad_leg(P, torch, args.seed, args.grad_batch, args.grad_K)
    if not args.no_phenom:
        result["phenomenological"] = phenom_leg(P, torch, args.seed, args.phenom_shots)
        result["code_capacity"] = code_capacity_leg(P, torch, args.seed)
    if not args.no_tune:
        result["tuning"] = tuning_leg(P, torch, args.seed)

    result["plain"] = None
    result["batched_over_plain"] = None
    if not args.no_plain:
        n_plain = min(args.plain_shots, B)
        pouts = (torch.empty((n_plain, words), dtype=torch.int64, device=dev),
                 torch.empty((n_plain, 1), dtype=torch.uint8, device=dev),
                 torch.empty((n_plain, 8), dtype=torch.int32, device=dev))
        G.decode(synd[:1], plain=True, out=tuple(o[:1] for o in pouts))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        G.decode(synd[:n_plain], plain=True, out=pouts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        same = bool(torch.equal(pouts[0], corr[:n_plain]))
        result["plain"] = {"shots": n_plain, "shots_per_s": round(n_plain / dt, 2),
                           "same_corrections_as_batched": same}
        result["batched_over_plain"] = round(shots_per_s / (n_plain / dt), 1)
        log(f"plain: {n_plain / dt:.2f} shots/s over {n_plain} shots; batched/plain "
            f"{result['batched_over_plain']}x; identical corrections: {same}")
    if not args.no_latency:
        nb, bs = args.latency_batches, args.latency_batch
        outs = (torch.empty((bs, words), dtype=torch.int64, device=dev),
                torch.empty((bs, 1), dtype=torch.uint8, device=dev),
                torch.empty((bs, 8), dtype=torch.int32, device=dev))
        G.decode(synd[:bs], out=outs)
        torch.cuda.synchronize()
        lat = []
        for i in range(nb):
            lo = (i * bs) % max(B - bs, 1)
            t1 = time.perf_counter()
            G.decode(synd[lo:lo + bs], out=outs)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
        lat = np.array(lat)
        result["latency"] = {"batch": bs, "batches": nb,
                             "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                             "shots_per_s": round(bs * nb / float(lat.sum()), 1)}
        result["p99_latency_ms"] = result["latency"]["p99_ms"]
        log(f"latency: p50 {result['latency']['p50_ms']} ms, p99 {result['latency']['p99_ms']} ms "
            f"per {bs}-shot batch")

    if not args.no_cpu:
        from oracle import oracle as O

        g = O.OracleGraph(dem)
        threads = min(16, os.cpu_count() or 1)
        done = 0
        t1 = time.perf_counter()
        chunk = threads * 2
        while time.perf_counter() - t1 < args.cpu_seconds and done + chunk <= B:
            O.decode(g, perms, batch.syndromes[done:done + chunk], L=L, M=M, T=T, alpha=alpha,
                     threads=threads)
            done += chunk
        dt = time.perf_counter() - t1
        # one thread on the next shots, for the per-core rate
        one, t2 = 0, time.perf_counter()
        while time.perf_counter() - t2 < args.cpu_seconds / 3 and done + one < B:
            O.decode(g, perms, batch.syndromes[done + one:done + one + 1], L=L, M=M, T=T, alpha=alpha, threads=1)
            one += 1
        dt1 = time.perf_counter() - t2
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        result["cpu_baseline"] = {"value": round(done / dt, 3), "unit": "shots/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"first {done} shots of the batch, {dt:.1f}s, "
                                            f"{threads} threads, FP64 oracle",
                                  "single_thread_value": round(one / dt1, 4) if one else None,
                                  "nproc": os.cpu_count(), "cpu_model": model}
        log(f"cpu oracle: {done / dt:.2f} shots/s on {threads} threads, {one / dt1:.3f} on one")

    print(json.dumps(result), flush=True)
    G.close()


if __name__ == "__main__":
    main()
