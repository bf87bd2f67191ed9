"""Pins of the oracle's tie witnesses, the values that decide which FP32
disagreements the GPU parity tests excuse.

  min_abs_post   the smallest |L_v| of any hard decision a member took
                 (Algorithm 1's decision e_v = 1 iff L_v <= 0); a decision
                 whose posterior lies within FP32 rounding of zero can go
                 either way, and with it the convergence iteration.
  min_gap        the smallest difference between the soft values of the
                 column LSD chose and the runner-up, over every rank
                 decision it took (Sec. III.C: each growth step's boundary
                 choice and the rank order of each cluster's columns).

Each expected value below is worked out by hand from the definitions, so a
witness computed over the wrong set (the chosen column instead of the
runner-up, the last round only, a signed instead of an absolute value) or
stuck at zero or infinity fails a case.  None of these tests uses the HIP
path.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth.dem import dem_from_dense


def _graph(H, priors):
    H = np.asarray(H, np.uint8)
    return O.OracleGraph(dem_from_dense(H, np.asarray(priors, float), np.ones((1, H.shape[1]), np.uint8)))


CHAIN = np.array([[1, 1, 0, 0, 0, 0],
                  [0, 1, 1, 0, 0, 0],
                  [0, 0, 1, 1, 0, 0],
                  [0, 0, 0, 1, 1, 0],
                  [0, 0, 0, 0, 1, 1]], np.uint8)


@pytest.mark.parametrize("flipped,q,gap", [
    # c1 takes v2 (q 1) over v1 (4): 3; c3 takes v3 (2) over v4 (3): 1; the
    # merged cluster orders v2 < v3: 1
    ([1, 3], [5, 4, 1, 2, 3, 6], 1.0),
    # c0 takes v0 (1) over v1 (5): 4; c4 takes v5 (2) over v4 (5): 3; both
    # clusters hold one column, so no ordering gap
    ([0, 4], [1, 5, 5, 5, 5, 2], 3.0),
    # growth gaps 8 and 5, then 7 and 6 (both clusters take v2); the merged
    # cluster orders v1 < v2 < v3 at gaps 1 and 1
    ([0, 3], [9, 1, 2, 3, 8, 9], 1.0),
    # v2 (3) over v3 (9): 6; then v1 and v3 tie at 9 (taken by index): 0
    ([2], [9, 9, 3, 9, 9, 9], 0.0),
    # as the first case with q scaled by 0.25 and shifted: gaps scale too
    ([1, 3], [1.25, 1.0, 0.25, 0.5, 0.75, 1.5], 0.25),
])
def test_lsd_min_gap_chain(flipped, q, gap):
    g = _graph(CHAIN, np.full(6, 0.1))
    s = np.zeros(5, np.uint8)
    s[flipped] = 1
    r = O.lsd(g, s, np.array(q, float))
    assert r["min_gap"] == gap


def test_lsd_min_gap_triangle():
    """The triangle of checks with pendant columns (c0: v0 v2 v3, c1: v0 v1
    v4, c2: v1 v2 v5), s = c1.  Growth takes v1 (q 0.0, runner-up v0 at
    1.0), v0 (1.0 over v2 at 2.5), v2 (2.5 over v5 at 3.25) and v5 (3.25 over
    v4 at 4.0): gaps 1, 1.5, 0.75, 0.75; the cluster's columns in rank order
    v1 v0 v2 v5 have gaps 1, 1.5, 0.75.  The smallest is 0.75."""
    TRI = np.array([[1, 0, 1, 1, 0, 0], [1, 1, 0, 0, 1, 0], [0, 1, 1, 0, 0, 1]], np.uint8)
    g = _graph(TRI, [0.2, 0.05, 0.2, 0.05, 0.2, 0.3])
    r = O.lsd(g, np.array([0, 1, 0], np.uint8), np.array([1.0, 0.0, 2.5, 5.0, 4.0, 3.25]))
    assert r["rounds"] == 4
    assert r["min_gap"] == 0.75


def test_lsd_min_gap_no_decision():
    """A zero syndrome takes no rank decision: the witness is infinite."""
    g = _graph(CHAIN, np.full(6, 0.1))
    r = O.lsd(g, np.zeros(5, np.uint8), np.arange(6, dtype=float))
    assert np.isinf(r["min_gap"])


def _single_check_posteriors(lam, s, alpha):
    """H = [1 ... 1]: L_v = lambda_v + (1 - 2s) alpha prod_{u != v} sign
    lambda_u min_{u != v} |lambda_u|, the same at every iteration."""
    out = []
    for v in range(len(lam)):
        others = np.delete(lam, v)
        out.append(lam[v] + (1 - 2 * s) * alpha * np.prod(np.sign(others)) * np.abs(others).min())
    return np.array(out)


@pytest.mark.parametrize("schedule", ["serial", "parallel", "layered"])
def test_min_abs_post_single_check(schedule):
    """The decision witness of one member on one check: min_v |L_v|, with L_v
    from the closed form (a negative posterior counts by its magnitude)."""
    lam = np.array([2.0, -0.5, 2.9, 0.8, 1.4])
    pri = 1.0 / (1.0 + np.exp(lam))
    g = _graph(np.ones((1, 5)), pri)
    lam = O.prior_llr(pri)
    want = np.abs(_single_check_posteriors(lam, 1, 0.625)).min()
    if schedule == "layered":
        r = O.bp_layered(g, np.array([1], np.uint8), np.array([0]), T=3, stop=False)
    else:
        r = O.bp(g, np.array([1], np.uint8), perm=np.array([3, 1, 4, 0, 2]) if schedule == "serial" else None,
                 T=3, stop=False)
    np.testing.assert_allclose(r["min_abs_post"], want, rtol=1e-14)
    # by hand: column 1 is the only negative LLR; its others all have sign
    # + and least magnitude 0.8, so L_1 = -0.5 - 0.625 * 0.8 = -1.0, while
    # every other column gains 0.625 * 0.5 (sign product -, s = 1): 2.3125,
    # 3.2125, 1.1125, 1.7125.  The smallest magnitude is |L_1| = 1.0.
    np.testing.assert_allclose(want, 1.0, rtol=1e-12)


def test_min_abs_post_serial_path_by_hand():
    """Path v0 - c0 - v1 - c1 - v2, s = (0, 1), alpha = 0.5, one serial
    sweep: L = (a + b/2, b + a/2 - c/2, c - (b + a/2)/2) with a, b, c the
    LLRs of priors 0.1, 0.2, 0.3; the smallest magnitude is |L_2|."""
    pri = np.array([0.1, 0.2, 0.3])
    a, b, c = np.log((1 - pri) / pri)
    g = _graph([[1, 1, 0], [0, 1, 1]], pri)
    r = O.bp(g, np.array([0, 1], np.uint8), perm=np.array([0, 1, 2]), T=1, alpha=0.5, stop=False)
    L = np.array([a + b / 2, b + a / 2 - c / 2, c - (b + a / 2) / 2])
    np.testing.assert_allclose(r["min_abs_post"], np.abs(L).min(), rtol=1e-13)
    assert abs(L[2]) < min(abs(L[0]), abs(L[1]))


def test_decode_witnesses_single_check():
    """The whole decoder on one check with s = 1 and LLRs (2.0, 2.2, 2.5, 3.0,
    1.5): every posterior is lambda_v - 0.625 min_{u != v} lambda_u > 0, so
    no member converges and LSD runs.  Both members hold the same
    posteriors L (the schedule of one check does not matter), so the
    normalised average is 2 L / ||L|| and LSD's first choice, column 4
    (L = 0.25), beats column 0 (L = 1.0625) by 2 (1.0625 - 0.25) / ||L||;
    the one-column cluster is then valid and has no ordering gap.  The
    decision witness is 0.25."""
    lam = np.array([2.0, 2.2, 2.5, 3.0, 1.5])
    pri = 1.0 / (1.0 + np.exp(lam))
    g = _graph(np.ones((1, 5)), pri)
    perms = np.array([[0, 1, 2, 3, 4], [4, 3, 2, 1, 0]], np.uint32)
    out = O.decode(g, perms, np.array([[1]], np.uint8), L=2, M=1, T=5, threads=1)
    assert out["lsd_used"][0] and not out["converged"][0]
    assert np.flatnonzero(out["ehat"][0]).tolist() == [4]
    L = lam - 0.625 * np.array([1.5, 1.5, 1.5, 1.5, 2.0])
    np.testing.assert_allclose(L, [1.0625, 1.2625, 1.5625, 2.0625, 0.25], rtol=1e-12)
    np.testing.assert_allclose(out["min_abs_post"][0], 0.25, rtol=1e-12)
    np.testing.assert_allclose(out["min_q_gap"][0], 2 * (1.0625 - 0.25) / np.linalg.norm(L), rtol=1e-12)
    assert np.isinf(out["w_gap"][0])


def test_decode_weight_gap():
    """A converged shot's weight witness is the gap between the chosen
    candidate's prior weight and the runner-up's among the first M.  One
    check, s = 1, LLRs (0.5, 3.0, 3.0, 3.0): column 0's posterior is
    0.5 - 0.625 * 3 < 0 and the others stay positive, so every member
    converges at t = 1 on e = {v0}; all candidates are equal and the gap is
    0."""
    lam = np.array([0.5, 3.0, 3.0, 3.0])
    pri = 1.0 / (1.0 + np.exp(lam))
    g = _graph(np.ones((1, 4)), pri)
    perms = np.array([[0, 1, 2, 3], [3, 2, 1, 0], [1, 0, 3, 2]], np.uint32)
    out = O.decode(g, perms, np.array([[1]], np.uint8), L=3, M=3, T=4, threads=1)
    assert out["converged"][0] and out["winner"][0] == 0 and out["t_win"][0] == 1
    assert np.flatnonzero(out["ehat"][0]).tolist() == [0]
    assert out["w_gap"][0] == 0.0


SAT_H = np.array([[1, 0, 0], [1, 0, 0], [0, 1, 1]], np.uint8)  # v0 in two checks of degree 1


@pytest.mark.parametrize("synd,alpha,flags", [
    # c0 and c1 unflipped: each sends +alpha * clamp to v0, so L_0 = lambda +
    # 1.25e6 reaches the clamp; c2 flipped cannot be met by BP (L_1, L_2 stay
    # positive): LSD runs, and a member saturated
    ([0, 0, 1], 0.625, 2 | 8),
    # c0 and c1 flipped: L_0 = lambda - 1.25e6 is clamped, e_0 = 1 converges
    # at t = 1, and the winner's run saturated
    ([1, 1, 0], 0.625, 1 | 8),
    # zero syndrome, every LLR positive: decided without running BP, no flag
    ([0, 0, 0], 0.625, 1),
    # c0 flipped, c1 not: the two saturated check messages cancel in L_0 and
    # every mu stays at |lambda +- 6.25e5| < 1e6; LSD cannot explain c0 alone
    ([1, 0, 0], 0.625, 2 | 4),
    # alpha = 0.3: 2 * 0.3e6 + lambda < 1e6, nothing saturates
    ([0, 0, 1], 0.3, 2),
    ([1, 1, 0], 0.3, 1),
])
def test_saturation_flag_by_hand(synd, alpha, flags):
    """The saturation witness (flag 8): a message or posterior reached the
    clamp, in the winner's run or, when LSD ran, in any member's."""
    g = _graph(SAT_H, np.full(3, 0.1))
    perms = np.array([[0, 1, 2], [2, 1, 0]], np.uint32)
    out = O.decode(g, perms, np.array([synd], np.uint8), L=2, M=1, T=4, alpha=alpha, threads=1)
    assert int(out["rec"][0, 0]) == flags
