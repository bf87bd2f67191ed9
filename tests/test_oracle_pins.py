"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Each test names the passage it follows and what a plausible mistake in the
oracle would break.  None of these tests uses the HIP path.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from synth.dem import (circuit_dem, code_capacity_dem, dem_from_dense, phenomenological_dem)
from synth.sample import permutations, sample


def _dem(H, priors, lobs=None):
    H = np.asarray(H, np.uint8)
    if lobs is None:
        lobs = np.ones((1, H.shape[1]), np.uint8)
    return dem_from_dense(H, priors, lobs)


def _random_forest(rng, n_vars, max_deg=4):
    """A Tanner forest: every check has degree >= 2, no cycles."""
    rows = []
    var_of = [0]  # variables created so far (ids)
    nv = 1
    while nv < n_vars:
        v = int(rng.choice(var_of))
        k = int(rng.integers(1, max_deg))  # new neighbours of a fresh check
        k = min(k, n_vars - nv)
        new = list(range(nv, nv + k))
        nv += k
        var_of += new
        rows.append([v] + new)
    H = np.zeros((len(rows), n_vars), np.uint8)
    for c, r in enumerate(rows):
        H[c, r] = 1
    return H


# ---------------------------------------------------------------------------
# min-sum BP (Algorithm 1)


@pytest.mark.parametrize("schedule", ["serial", "parallel"])
@pytest.mark.parametrize("seed", range(6))
def test_tree_min_sum_equals_min_marginals(schedule, seed):
    """P1: on a forest, min-sum (alpha = 1) is max-product in the log domain,
    so after enough iterations L_v = W_1(v) - W_0(v) exactly (Algorithm 1's
    updates; the syndrome sign of syndrome-based decoding).  A wrong sign,
    a dropped extrinsic term or a min that includes the receiver breaks it."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 13))
    H = _random_forest(rng, n)
    pri = rng.uniform(0.02, 0.45, n)
    e = (rng.random(n) < 0.3).astype(np.uint8)
    s = (H.astype(int) @ e % 2).astype(np.uint8)
    dem = _dem(H, pri)
    g = O.OracleGraph(dem)
    lam = O.prior_llr(pri)
    perm = rng.permutation(n) if schedule == "serial" else None
    T = 2 * (n + H.shape[0])
    r = O.bp(g, s, perm=perm, T=T, alpha=1.0, stop=False)
    W = brute.min_weight_marginals(H, lam, s)
    np.testing.assert_allclose(r["post"], W[:, 1] - W[:, 0], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s", [0, 1])
def test_single_check_closed_form(s):
    """P2: H = [1 ... 1]: every variable has one check, so its outgoing
    message stays lambda_v and L_v = lambda_v + (1-2s) alpha prod_{u!=v}
    sign(lambda_u) min_{u!=v} |lambda_u| at every iteration."""
    pri = np.array([0.1, 0.7, 0.05, 0.3, 0.2])
    lam = O.prior_llr(pri)
    dem = _dem(np.ones((1, 5)), pri)
    g = O.OracleGraph(dem)
    alpha = 0.625
    r = O.bp(g, np.array([s]), perm=np.array([3, 1, 4, 0, 2]), T=4, alpha=alpha, stop=False,
             trace=True)
    for v in range(5):
        others = [u for u in range(5) if u != v]
        sg = np.prod(np.sign(lam[others]))
        exp = lam[v] + (1 - 2 * s) * alpha * sg * np.min(np.abs(lam[others]))
        np.testing.assert_allclose(r["trace"][:, v], exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("schedule", ["serial", "parallel"])
def test_single_check_per_iteration_scaling(schedule):
    """P2 with a scaling factor per iteration: on H = [1 ... 1] the posterior
    after iteration t is lambda_v + (1-2s) alpha_t prod sign min, so each
    row of the trace carries its own alpha_t.  Breaks on an iteration index
    off by one or a factor taken from the wrong end of the list."""
    pri = np.array([0.1, 0.7, 0.05, 0.3, 0.2])
    lam = O.prior_llr(pri)
    g = O.OracleGraph(_dem(np.ones((1, 5)), pri))
    alpha = np.array([0.9, 0.5, 0.75, 0.3])
    perm = np.array([3, 1, 4, 0, 2]) if schedule == "serial" else None
    r = O.bp(g, np.array([1]), perm=perm, T=4, alpha=alpha, stop=False, trace=True)
    for v in range(5):
        others = [u for u in range(5) if u != v]
        sg = np.prod(np.sign(lam[others]))
        exp = lam[v] - alpha * sg * np.min(np.abs(lam[others]))
        np.testing.assert_allclose(r["trace"][:, v], exp, rtol=0, atol=1e-15)


def test_serial_first_iteration_by_hand():
    """Algorithm 1, serial branch: a column updated later in the sweep sees
    messages already refreshed earlier in the same sweep; the parallel branch
    does not.  Path v0 - c0 - v1 - c1 - v2, s = (0, 1), alpha = 0.5."""
    pri = np.array([0.1, 0.2, 0.3])
    a, b, c = O.prior_llr(pri)
    H = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    g = O.OracleGraph(_dem(H, pri))
    s = np.array([0, 1], np.uint8)
    al = 0.5
    ser = O.bp(g, s, perm=np.array([0, 1, 2]), T=1, alpha=al, stop=False)["post"]
    # v0: r_{c0->v0} = al*b
    L0 = a + al * b
    # v1: r_{c0->v1} = al*|mu_{v0->c0}| = al*a ; r_{c1->v1} = -al*c
    L1 = b + al * a - al * c
    mu_v1_c1 = b + al * a
    # v2: r_{c1->v2} = -al*mu_{v1->c1} (fresh)
    L2 = c - al * mu_v1_c1
    np.testing.assert_allclose(ser, [L0, L1, L2], rtol=0, atol=1e-14)
    par = O.bp(g, s, perm=None, T=1, alpha=al, stop=False)["post"]
    np.testing.assert_allclose(par, [a + al * b, b + al * a - al * c, c - al * b], rtol=0,
                               atol=1e-14)


def _levels(dem, perm):
    cols = dem.column_lists()
    last = np.zeros(dem.m, np.int64)
    lev = np.zeros(dem.n, np.int64)
    for v in perm:
        lv = 1 + max((last[c] for c in cols[v]), default=0)
        lev[v] = lv
        for c in cols[v]:
            last[c] = lv
    return lev


@pytest.mark.parametrize("which", ["phenom", "circuit"])
def test_serial_level_order_is_bitwise_identical(which):
    """P3: two columns that share no check commute exactly under the serial
    schedule, so executing the schedule level by level (any linear extension
    of its dependency order) gives bit-identical FP64 posteriors."""
    dem = phenomenological_dem(5, 3, 0.05, 0.05) if which == "phenom" else circuit_dem(3, 2, 0.01)
    g = O.OracleGraph(dem)
    rng = np.random.default_rng(7)
    perm = rng.permutation(dem.n)
    lev = _levels(dem, perm)
    # stable sort by level, then reverse inside each level
    order = sorted(range(dem.n), key=lambda k: (lev[perm[k]], -k))
    perm2 = perm[order]
    b = sample(dem, 5, 3)
    for s in b.syndromes:
        r1 = O.bp(g, s, perm=perm, T=6, stop=False, trace=True)
        r2 = O.bp(g, s, perm=perm2, T=6, stop=False, trace=True)
        assert np.array_equal(r1["trace"], r2["trace"])
    # swaps of columns that do share a check are not invisible in general
    cols = dem.column_lists()
    differs = False
    tried = 0
    for k in range(dem.n - 1):
        if not set(cols[perm[k]]) & set(cols[perm[k + 1]]):
            continue
        perm3 = perm.copy()
        perm3[k], perm3[k + 1] = perm3[k + 1], perm3[k]
        for s in b.syndromes:
            r1 = O.bp(g, s, perm=perm, T=3, stop=False, trace=True)
            r3 = O.bp(g, s, perm=perm3, T=3, stop=False, trace=True)
            differs |= not np.array_equal(r1["trace"], r3["trace"])
        tried += 1
        if differs or tried > 20:
            break
    assert differs


# ---------------------------------------------------------------------------
# the whole decoder on the Steane / d=3 colour code


def test_steane_exhaustive_against_ml():
    """P5: the d=3 6.6.6 code is the Steane code.  Decoding all 2^7 errors:
    every output satisfies H e = s (LSD always returns a syndrome-consistent
    correction, paper Sec. III.C), every weight <= 1 error lands in the right
    coset, and the exact failure probability is at least the ML one."""
    p = 0.05
    dem = code_capacity_dem(3, p)
    H, Lo = dem.dense_h(), dem.dense_l()
    g = O.OracleGraph(dem)
    E = brute.all_errors(7)
    S = (E.astype(int) @ H.T % 2).astype(np.uint8)
    out = O.decode(g, permutations(7, 16, 5), S, L=16, M=5, T=32)
    assert np.array_equal(out["ehat"].astype(int) @ H.T % 2, S)
    true_obs = (E.astype(int) @ Lo.T % 2).astype(np.uint8)
    w = E.sum(1)
    assert np.array_equal(out["obs"][w <= 1], true_obs[w <= 1])
    prob = np.prod(np.where(E == 1, p, 1 - p), axis=1)
    fail = prob[(out["obs"] != true_obs).any(1)].sum()
    _, ml_fail = brute.ml_coset_table(H, Lo, np.full(7, p))
    assert fail >= ml_fail - 1e-15
    # ML corrects every single error, so its failure is O(p^2)
    assert ml_fail < 30 * p * p


def test_code_capacity_d5_vs_ml():
    """P6 (bounds only): VibeLSD is not ML, so on the d=5 code its logical
    failure rate over sampled shots is not below ML's (up to sampling
    error), and it agrees with ML's choice on the vast majority of shots."""
    p = 0.05
    dem = code_capacity_dem(5, p)
    H, Lo = dem.dense_h(), dem.dense_l()
    table, ml_fail = brute.ml_coset_table(H, Lo, dem.priors)
    b = sample(dem, 4000, 11)
    g = O.OracleGraph(dem)
    out = O.decode(g, permutations(dem.n, 16, 3), b.syndromes, L=16, M=5, T=32)
    assert np.array_equal(out["ehat"].astype(int) @ H.T % 2, b.syndromes)
    ml_obs = np.array([table[bytes(s)] for s in b.syndromes], np.uint8)
    agree = (ml_obs == out["obs"]).all(1).mean()
    assert agree > 0.97
    ler = (out["obs"] != b.observables).any(1).mean()
    sigma = np.sqrt(ml_fail * (1 - ml_fail) / len(b.syndromes))
    assert ler >= ml_fail - 4 * sigma


# ---------------------------------------------------------------------------
# selection and averaging (Sec. III.D.2)


def test_selection_is_min_weight_over_first_M():
    """P11: the winner is the minimum-prior-weight candidate among the first
    M converged members in (iteration, index) order; with M >= L it is the
    minimum over every converged member, and relabelling the members (with
    their schedules) does not change it."""
    dem = phenomenological_dem(5, 3, 0.04, 0.04)
    g = O.OracleGraph(dem)
    lam = O.prior_llr(dem.priors)
    L, T = 12, 15
    perms = permutations(dem.n, L, 9)
    b = sample(dem, 40, 21)
    for M in (3, L):
        out = O.decode(g, perms, b.syndromes, L=L, M=M, T=T, want_members=True)
        for sh in range(len(b.syndromes)):
            runs = [O.bp(g, b.syndromes[sh], perm=perms[i], T=T) for i in range(L)]
            tc = np.array([r["t_conv"] for r in runs])
            assert np.array_equal(tc, out["t_members"][sh])
            conv = [i for i in range(L) if tc[i] > 0]
            if not conv:
                assert out["lsd_used"][sh]
                continue
            first = sorted(conv, key=lambda i: (tc[i], i))[:M]
            w = [float(runs[i]["ehat"].astype(np.float64) @ lam) for i in first]
            best = first[int(np.argmin(w))]
            assert out["winner"][sh] == best
            assert np.array_equal(out["ehat"][sh], runs[best]["ehat"])
    rng = np.random.default_rng(1)
    lab = rng.permutation(L)
    a = O.decode(g, perms, b.syndromes, L=L, M=L, T=T)
    c = O.decode(g, perms[lab], b.syndromes, L=L, M=L, T=T)
    amb = a["w_gap"] == 0  # exact weight ties are broken by member label
    assert np.array_equal(a["ehat"][~amb], c["ehat"][~amb])


def test_normalised_average_closed_form():
    """P12: with no member converged, q = (1/L) sum_i LLR^i / ||LLR^i||_2
    over the members' final posteriors (Sec. III.D.2), to within the 2^-57
    rounding of each term."""
    dem = circuit_dem(3, 2, 0.02)
    g = O.OracleGraph(dem)
    L, T = 6, 2
    perms = permutations(dem.n, L, 4)
    b = sample(dem, 200, 5)
    out = O.decode(g, perms, b.syndromes, L=L, M=2, T=T, want_q=True)
    idx = np.flatnonzero(out["lsd_used"])
    assert len(idx) > 0
    for sh in idx[:5]:
        posts = [O.bp(g, b.syndromes[sh], perm=perms[i], T=T, stop=False)["post"]
                 for i in range(L)]
        q = sum(p / np.linalg.norm(p) for p in posts) / L
        np.testing.assert_allclose(out["q"][sh], q, rtol=1e-12, atol=1e-15)
        # LSD only uses the order of q: a positive rescale changes nothing
        r1 = O.lsd(g, b.syndromes[sh], q)
        r2 = O.lsd(g, b.syndromes[sh], 3.5 * q)
        assert np.array_equal(r1["ehat"], r2["ehat"])
    # the average is summed exactly in 2^-56 fixed point: reversing the order
    # of the members leaves q bit-identical on every shot that reaches LSD,
    # and with it the LSD correction
    rev = O.decode(g, perms[::-1].copy(), b.syndromes, L=L, M=2, T=T, want_q=True)
    assert np.array_equal(rev["lsd_used"], out["lsd_used"])
    assert np.array_equal(rev["q"][idx], out["q"][idx])
    assert np.array_equal(rev["ehat"][idx], out["ehat"][idx])


# ---------------------------------------------------------------------------
# LSD-0 (Sec. III.C)

CHAIN = np.array([[1, 1, 0, 0, 0, 0],
                  [0, 1, 1, 0, 0, 0],
                  [0, 0, 1, 1, 0, 0],
                  [0, 0, 0, 1, 1, 0],
                  [0, 0, 0, 0, 1, 1]], np.uint8)


@pytest.mark.parametrize("case", [
    # flipped checks, q, expected clusters as (checks, bits), rounds, correction
    ([1, 3], [5, 4, 1, 2, 3, 6], [({1, 2, 3}, {2, 3})], 1, {2, 3}),
    ([0, 4], [1, 5, 5, 5, 5, 2], [({0}, {0}), ({4}, {5})], 1, {0, 5}),
    ([0, 3], [9, 1, 2, 3, 8, 9], [({0, 1, 2, 3}, {1, 2, 3})], 2, {1, 2, 3}),
    # an isolated defect: v2 alone leaves c1 unexplained; the q tie between v1
    # and v3 goes to the lower index; v0 then closes the cluster
    ([2], [9, 9, 3, 9, 9, 9], [({0, 1, 2}, {0, 1, 2})], 3, {0, 1, 2}),
])
def test_lsd_hand_worked_chain(case):
    """P9: hand-worked cluster growth on a repetition chain (each column joins
    two neighbouring checks, the end columns one): one column per invalid
    cluster per round, the lowest-q boundary column, merge on shared checks,
    stop when every cluster is valid."""
    flipped, q, clusters, rounds, corr = case
    g = O.OracleGraph(_dem(CHAIN, np.full(6, 0.1)))
    s = np.zeros(5, np.uint8)
    s[flipped] = 1
    r = O.lsd(g, s, np.array(q, float))
    assert not r["failed"]
    assert r["rounds"] == rounds
    got = []
    for lab in range(r["clusters"]):
        got.append((set(np.flatnonzero(r["check_label"] == lab).tolist()),
                    set(np.flatnonzero(r["bit_label"] == lab).tolist())))
    key = lambda kv: min(kv[0])
    assert sorted(got, key=key) == sorted(clusters, key=key)
    assert set(np.flatnonzero(r["ehat"]).tolist()) == corr


def test_lsd_fails_outside_image():
    """A flipped check with no columns cannot be explained: the cluster has an
    empty boundary and LSD reports failure with no correction for it."""
    H = np.array([[1, 1], [0, 0]], np.uint8)
    g = O.OracleGraph(_dem(H, [0.1, 0.1]))
    r = O.lsd(g, np.array([0, 1], np.uint8), np.array([0.0, 0.0]))
    assert r["failed"] and not r["ehat"].any()


@pytest.mark.parametrize("seed", range(4))
def test_lsd_cluster_invariants_and_osd0(seed):
    """P4, P7-P9 on random soft inputs over a small circuit-level DEM: the
    output satisfies H e = s; clusters are disjoint, cover every flipped check,
    contain every check of their columns, are valid; and each cluster's
    solution is the unique one on the greedy GF(2) basis of its columns taken
    in (q, index) order (OSD-0 on the cluster), found here by enumeration."""
    dem = circuit_dem(3, 2, 0.01)
    H = dem.dense_h()
    g = O.OracleGraph(dem)
    rng = np.random.default_rng(seed)
    b = sample(dem, 30, 100 + seed)
    for s in b.syndromes:
        if not s.any():
            continue
        q = rng.normal(size=dem.n)
        r = O.lsd(g, s, q)
        assert not r["failed"]
        assert np.array_equal(H.astype(int) @ r["ehat"] % 2, s)
        cl, bl = r["check_label"], r["bit_label"]
        assert np.all(cl[s == 1] >= 0)
        for v in np.flatnonzero(bl >= 0):
            assert np.all(cl[H[:, v] == 1] == bl[v])
        for lab in range(r["clusters"]):
            rows = np.flatnonzero(cl == lab)
            cols = np.flatnonzero(bl == lab)
            A = H[np.ix_(rows, cols)]
            assert brute.gf2_in_span(A, s[rows])
            if len(cols) > 18:
                continue
            order = sorted(range(len(cols)), key=lambda j: (q[cols[j]], cols[j]))
            piv = brute.greedy_basis(A, order)
            x = brute.solve_on(A, piv, s[rows])
            assert np.array_equal(x, r["ehat"][cols])
