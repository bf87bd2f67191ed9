"""Pins of the oracle's higher-order LSD (the combination sweep over each
cluster's non-pivot columns, weighted by the prior LLRs).

The paper runs LSD-0, the variant that leaves out the higher-order search
around the first solution (Sec. III.D.1 step 5), and cites OSD, whose
combination sweep that search is (Sec. III.C); the workload list
asks for order 10 on the phenomenological workload.  The sweep is the
ordered-statistics combination sweep: no non-pivot column, each single
non-pivot column, each pair among the first `order` of them (rank order);
pivots re-solved for each; least prior weight wins, ties to the earlier.
"""
import itertools

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from synth.dem import circuit_dem, dem_from_dense
from synth.sample import sample

# A triangle of checks with one pendant column per check:
#   c0: v0 v2 v3   c1: v0 v1 v4   c2: v1 v2 v5     (v0 + v1 + v2 = 0)
TRI = np.array([[1, 0, 1, 1, 0, 0], [1, 1, 0, 0, 1, 0], [0, 1, 1, 0, 0, 1]], np.uint8)


def _tri(priors):
    return O.OracleGraph(dem_from_dense(TRI, np.array(priors, float), np.ones((1, 6), np.uint8)))


def test_hand_worked_triangle():
    """s = c1, soft values rank v1 < v0 < v2 < v5 < v4 < v3.  Growth from
    c1 takes v1 (c1 alone is not explained), v0, v2 (dependent: v2 = v0 + v1)
    and v5, after which c1 = v1 + v5 is explained: 4 rounds, one cluster of
    v0 v1 v2 v5.  In rank order the pivots are v1, v0, v5 and v2 is the only
    non-pivot.  OSD-0 gives {v1, v5}.  The sweep's one further candidate sets
    v2: then c1 + v2's checks = c0 + c1 + c2 = v0 + v5, so e = {v0, v2, v5}.
    With priors (0.2, 0.05, 0.2, 0.05, 0.2, 0.3) the weights are
    ln 19 + ln(7/3) = 3.79 for OSD-0 and 2 ln 4 + ln(7/3) = 3.62 for the
    candidate, which wins; with p(v1) = 0.2 instead, OSD-0 weighs
    ln 4 + ln(7/3) = 2.23 and stays."""
    s = np.array([0, 1, 0], np.uint8)
    q = np.array([1.0, 0.0, 2.0, 5.0, 4.0, 3.0])
    g = _tri([0.2, 0.05, 0.2, 0.05, 0.2, 0.3])
    r0 = O.lsd(g, s, q)
    assert r0["rounds"] == 4 and r0["clusters"] == 1
    assert np.flatnonzero(r0["bit_label"] >= 0).tolist() == [0, 1, 2, 5]
    assert np.flatnonzero(r0["ehat"]).tolist() == [1, 5]
    for order in (1, 2, 10):
        r = O.lsd(g, s, q, order=order)
        assert np.flatnonzero(r["ehat"]).tolist() == [0, 2, 5]
        assert (r["clusters"], r["largest"], r["rounds"]) == (r0["clusters"], r0["largest"], r0["rounds"])
    g2 = _tri([0.2, 0.2, 0.2, 0.05, 0.2, 0.3])
    assert np.flatnonzero(O.lsd(g2, s, q, order=1)["ehat"]).tolist() == [1, 5]


def _weight(lam, x):
    return float(np.sum(lam[x.astype(bool)]))


@pytest.mark.parametrize("seed", range(3))
def test_small_clusters_reach_the_minimum_weight_solution(seed):
    """On a cluster with at most two non-pivot columns and order >= 2, the
    candidates set every subset of the non-pivot columns, and each subset
    fixes one solution: the sweep returns the least-weight solution of the
    cluster's checks over its columns, found here by enumerating every
    assignment of the columns.  On every cluster, any order: the output
    solves the cluster's checks, and its weight never exceeds that of a
    lower order (the candidate sets are nested).  Breaks on a candidate
    solved without the chosen columns' syndrome, a weight taken from the
    soft values, or a comparison keeping the heavier candidate."""
    dem = circuit_dem(3, 2, 0.01)
    H = dem.dense_h()
    g = O.OracleGraph(dem)
    lam = O.prior_llr(dem.priors)
    rng = np.random.default_rng(seed)
    b = sample(dem, 40, 200 + seed)
    pinned = 0
    for s in b.syndromes:
        if not s.any():
            continue
        q = rng.normal(size=dem.n)
        res = {o: O.lsd(g, s, q, order=o) for o in (0, 1, 2, 10)}
        bl, cl = res[0]["bit_label"], res[0]["check_label"]
        for o in (1, 2, 10):
            assert np.array_equal(res[o]["bit_label"], bl)
        for lab in range(res[0]["clusters"]):
            rows = np.flatnonzero(cl == lab)
            cols = np.flatnonzero(bl == lab)
            A = H[np.ix_(rows, cols)].astype(np.int64)
            w = {o: _weight(lam[cols], res[o]["ehat"][cols]) for o in res}
            for o in (0, 1, 2, 10):
                assert np.array_equal(A @ res[o]["ehat"][cols] % 2, s[rows])
            assert w[1] <= w[0] and w[2] <= w[1] and w[10] <= w[2]
            nf = len(cols) - brute.gf2_rank(A)
            if not (1 <= nf <= 2) or len(cols) > 16:
                continue
            X = np.array(list(itertools.product((0, 1), repeat=len(cols))), np.int64)
            sol = X[np.all(X @ A.T % 2 == s[rows], axis=1)]
            assert len(sol) == 2 ** nf
            ws = sol @ lam[cols]
            order = np.argsort(ws)
            if ws[order[1]] - ws[order[0]] < 1e-9:
                continue
            assert np.array_equal(res[2]["ehat"][cols], sol[order[0]])
            assert np.array_equal(res[10]["ehat"][cols], sol[order[0]])
            pinned += 1
    assert pinned >= 5, pinned
