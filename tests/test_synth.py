"""Input generators: colour code geometry, DEM shapes, sampler."""
import os

import numpy as np
import pytest

from oracle import brute
from synth.colour_code import triangular_666
from synth.dem import circuit_dem, code_capacity_dem, phenomenological_dem
from synth.sample import permutations, sample

GOLD = os.path.join(os.path.dirname(__file__), "golden", "colour_code_counts.txt")


def _rows():
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            yield [int(x) for x in line.split()]


@pytest.mark.parametrize("row", list(_rows()), ids=lambda r: f"d{r[0]}")
def test_colour_code_counts(row):
    d, n, P, w4, nnz, corner, edge, bulk = row
    code = triangular_666(d)
    H = code.check_matrix()
    assert code.n == n and H.shape == (P, n) and P == (n - 1) // 2
    w = H.sum(1)
    assert set(w.tolist()) <= {4, 6} and (w == 4).sum() == w4
    assert H.sum() == nnz
    deg = H.sum(0)
    assert [(deg == 1).sum(), (deg == 2).sum(), (deg == 3).sum()] == [corner, edge, bulk]
    # X and Z checks on the same plaquettes commute; n - 1 independent checks
    assert not (H.astype(int) @ H.T.astype(int) % 2).any()
    assert brute.gf2_rank(H) == P
    # the all-ones observable commutes with every check and is a logical
    assert not (H.sum(1) % 2).any() and n % 2 == 1


@pytest.mark.parametrize("d", [3, 5])
def test_colour_code_distance(d):
    """Smallest undetectable error with odd overlap with the all-ones logical
    has weight d (brute force)."""
    H = triangular_666(d).check_matrix().astype(np.int64)
    n = H.shape[1]
    E = brute.all_errors(n).astype(np.int64)
    ok = ~(E @ H.T % 2).any(1) & (E.sum(1) % 2 == 1)
    assert E[ok].sum(1).min() == d


def test_cnot_slots_distinct():
    code = triangular_666(9)
    seen = {}
    for members in code.plaquettes:
        for q, slot in members:
            assert (q, slot) not in seen
            seen[(q, slot)] = 1


def test_phenomenological_shape():
    dem = phenomenological_dem(11, 11, 0.01, 0.01)
    assert (dem.m, dem.n, dem.nnz) == (540, 1496, 3630)
    rd = np.diff(dem.h_indptr.astype(int))
    assert rd[-45:].tolist() == [1] * 45  # final perfect round: one column each
    L = dem.dense_l()[0]
    assert L[:1001].all() and not L[1001:].any()


def test_circuit_dem_shape_and_merge():
    dem, st = circuit_dem(9, 9, 1e-3, return_stats=True)
    assert dem.m == 540  # (n-1) detectors per round, 9 rounds
    cols = dem.column_lists()
    assert len(set(map(tuple, cols))) + 0 <= dem.n
    # merged mechanisms: no two columns share (detectors, observable)
    obs = dem.dense_l()[0]
    keys = {(tuple(c), int(o)) for c, o in zip(cols, obs)}
    assert len(keys) == dem.n
    assert max(len(c) for c in cols) <= 12 and min(len(c) for c in cols) >= 1
    # idling ancillas accumulate several faults into one mechanism
    assert np.all((dem.priors > 0) & (dem.priors < 0.05))
    assert st["elementary_faults"] > dem.n


def test_sampler_reproducible_and_consistent():
    dem = code_capacity_dem(5, 0.05)
    a = sample(dem, 3000, 42)
    b = sample(dem, 3000, 42)
    c = sample(dem, 3000, 43)
    assert np.array_equal(a.syndromes, b.syndromes)
    assert not np.array_equal(a.syndromes, c.syndromes)
    e = a.errors_dense(dem.n)
    assert np.array_equal(e.astype(int) @ dem.dense_h().T % 2, a.syndromes)
    assert np.array_equal(e.astype(int) @ dem.dense_l().T % 2, a.observables)
    # column firing rate matches the prior (binomial, 5 sigma)
    rate = e.mean(0)
    assert np.all(np.abs(rate - 0.05) < 5 * np.sqrt(0.05 * 0.95 / 3000))


def test_permutations():
    p = permutations(100, 8, 1)
    assert p.shape == (8, 100) and p.dtype == np.uint32
    for row in p:
        assert sorted(row.tolist()) == list(range(100))
    assert np.array_equal(p, permutations(100, 8, 1))


def test_circuit_dem_si1000_same_faults_table_rates():
    """Si1000 (Sec. IV.A table) changes the rates, not the circuit: the same
    elementary fault locations and the same merged columns as Uniform.  To
    first order a column's prior is the sum of its faults' rates, and each
    Si1000 rate is between 1/10 (idling in a gate layer) and 5 (readout
    flips) times the Uniform one, so every column's ratio lies in that range;
    columns made only of two-qubit gate faults keep their prior (ratio 1),
    and columns holding readout flips rise well above it."""
    u, su = circuit_dem(5, 5, 1e-4, return_stats=True)
    s, ss = circuit_dem(5, 5, 1e-4, return_stats=True, noise="si1000")
    assert su["elementary_faults"] == ss["elementary_faults"]
    assert u.m == s.m and u.n == s.n
    assert np.array_equal(u.dense_h(), s.dense_h()) and np.array_equal(u.dense_l(), s.dense_l())
    ratio = s.priors / u.priors
    assert ratio.min() >= 0.1 * (1 - 1e-3) and ratio.max() <= 5.0 * (1 + 1e-3)
    assert np.isclose(np.median(ratio), 1.0, rtol=1e-3)
    assert ratio.max() > 2.5 and ratio.min() < 0.5
    with pytest.raises(ValueError):
        circuit_dem(3, 3, 1e-3, noise="nope")
