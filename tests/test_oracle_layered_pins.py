"""Pins of the oracle's layered (check-serial) schedule, or_bp_layered.

The paper names layered schedules only as future work (Sec. V); the reading
is the usual layered form of min-sum: checks one at a time in a per-member
order, each from the latest posteriors, mu = L - r_own.  These pins check
it against facts that do not go through the oracle's code.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from synth.dem import code_capacity_dem, dem_from_dense
from synth.sample import permutations, sample


def _dem(H, priors):
    H = np.asarray(H, np.uint8)
    return dem_from_dense(H, priors, np.ones((1, H.shape[1]), np.uint8))


def _random_forest(rng, n_vars, max_deg=4):
    rows, var_of, nv = [], [0], 1
    while nv < n_vars:
        v = int(rng.choice(var_of))
        k = min(int(rng.integers(1, max_deg)), n_vars - nv)
        new = list(range(nv, nv + k))
        nv += k
        var_of += new
        rows.append([v] + new)
    H = np.zeros((len(rows), n_vars), np.uint8)
    for c, r in enumerate(rows):
        H[c, r] = 1
    return H


@pytest.mark.parametrize("seed", range(6))
def test_layered_tree_equals_min_marginals(seed):
    """On a forest min-sum with alpha = 1 is max-product in the log domain
    under any schedule, so after enough sweeps L_v = W_1(v) - W_0(v), the
    enumerated min-weight marginals.  Breaks on a wrong sign, on mu taken
    with the check's own message (L instead of L - r), or on a stale L."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(6, 13))
    H = _random_forest(rng, n)
    pri = rng.uniform(0.02, 0.45, n)
    e = (rng.random(n) < 0.3).astype(np.uint8)
    s = (H.astype(int) @ e % 2).astype(np.uint8)
    g = O.OracleGraph(_dem(H, pri))
    lam = O.prior_llr(pri)
    cperm = rng.permutation(H.shape[0])
    r = O.bp_layered(g, s, cperm, T=2 * (n + H.shape[0]), alpha=1.0, stop=False)
    W = brute.min_weight_marginals(H, lam, s)
    np.testing.assert_allclose(r["post"], W[:, 1] - W[:, 0], rtol=1e-12, atol=1e-12)


def test_layered_two_checks_by_hand():
    """Path v0 - c0 - v1 - c1 - v2, s = (0, 1), alpha = 0.5, order (c0, c1),
    one sweep.  c0 sees lambda: r00 = al*b, r01 = al*a.  c1 then sees
    v1's updated posterior b + al*a (c0's fresh message), so
    r12 = -al*(b + al*a) and r11 = -al*c.  In the order (c1, c0) the roles
    swap; a parallel sweep would give neither."""
    pri = np.array([0.1, 0.2, 0.3])
    a, b, c = O.prior_llr(pri)
    H = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    g = O.OracleGraph(_dem(H, pri))
    s = np.array([0, 1], np.uint8)
    al = 0.5
    p01 = O.bp_layered(g, s, np.array([0, 1]), T=1, alpha=al, stop=False)["post"]
    np.testing.assert_allclose(p01, [a + al * b, b + al * a - al * c, c - al * (b + al * a)], rtol=0, atol=1e-14)
    p10 = O.bp_layered(g, s, np.array([1, 0]), T=1, alpha=al, stop=False)["post"]
    # c1 first: r11 = -al*c, r12 = -al*b; then c0 sees v1 at b - al*c
    np.testing.assert_allclose(p10, [a + al * (b - al * c), b - al * c + al * a, c - al * b], rtol=0, atol=1e-14)


def test_layered_second_sweep_removes_own_message():
    """Single check H = [1 1 1]: in the second sweep mu_v must be
    L_v - r_v = lambda_v again (the check's own message removed), so every
    sweep gives the same posteriors; a mu that kept r_v would drift."""
    pri = np.array([0.1, 0.3, 0.2])
    lam = O.prior_llr(pri)
    g = O.OracleGraph(_dem(np.ones((1, 3)), pri))
    r = O.bp_layered(g, np.array([1], np.uint8), np.array([0]), T=3, alpha=0.625, stop=False, trace=True)
    for v in range(3):
        others = [u for u in range(3) if u != v]
        exp = lam[v] - 0.625 * np.prod(np.sign(lam[others])) * np.min(np.abs(lam[others]))
        np.testing.assert_allclose(r["trace"][:, v], exp, rtol=0, atol=1e-14)


def test_layered_commuting_checks_any_order():
    """Checks that share no column commute: on code capacity d = 5 the
    checks of one colour share no qubit, so swapping two of them inside the
    order changes nothing, bit for bit."""
    dem = code_capacity_dem(5, 0.05)
    g = O.OracleGraph(dem)
    H = dem.dense_h()
    b = sample(dem, 6, 3)
    cperm = permutations(dem.m, 1, 4)[0]
    # two adjacent positions whose checks share no column
    for i in range(dem.m - 1):
        if not (H[cperm[i]] & H[cperm[i + 1]]).any():
            break
    else:
        pytest.skip("no commuting neighbours in this order")
    sw = cperm.copy()
    sw[i], sw[i + 1] = sw[i + 1], sw[i]
    for s in b.syndromes:
        r1 = O.bp_layered(g, s, cperm, T=6, stop=False, trace=True)
        r2 = O.bp_layered(g, s, sw, T=6, stop=False, trace=True)
        assert np.array_equal(r1["trace"], r2["trace"])
