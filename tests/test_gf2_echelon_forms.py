"""The GF(2) elimination of LSD (Sec. III.C: a cluster is valid when its
syndrome lies in the span of its columns; the solution on the pivot
columns) done two ways on random column sets: in insertion order, with each
new vector reduced by the earlier ones one at a time (as the oracle does),
and with the basis kept in reduced echelon form, where a reduction xors the
vectors whose pivot bit is set in the input, in any order, and a new vector
clears its pivot from the earlier ones (as the LSD kernel does).  A span
element is fixed by its bits at the pivots, so both must give the same
reduced vectors, the same pivots, the same span tests and the same pivot
combinations (solutions and non-pivot representations).  Host-only model
of the two procedures; no GPU."""
import numpy as np
import pytest


def lowest(x):
    nz = np.flatnonzero(x)
    return int(nz[0]) if len(nz) else -1


class Insertion:
    def __init__(self, m):
        self.vecs, self.combs, self.piv = [], [], []
        self.m = m

    def reduce(self, x, comb):
        x, comb = x.copy(), comb.copy()
        for v, c, p in zip(self.vecs, self.combs, self.piv):
            if x[p]:
                x ^= v
                comb ^= c
        return x, comb

    def append(self, x, comb, p):
        self.vecs.append(x.copy())
        self.combs.append(comb.copy())
        self.piv.append(p)


class Reduced(Insertion):
    def reduce(self, x, comb):
        hits = [j for j, p in enumerate(self.piv) if x[p]]  # decided on the input alone
        x, comb = x.copy(), comb.copy()
        for j in reversed(hits):  # any order
            x ^= self.vecs[j]
            comb ^= self.combs[j]
        return x, comb

    def append(self, x, comb, p):
        for j in range(len(self.vecs)):
            if self.vecs[j][p]:
                self.vecs[j] ^= x
                self.combs[j] ^= comb
        super().append(x, comb, p)
        for j, pj in enumerate(self.piv):  # the form the reduction relies on
            assert all(self.vecs[k][pj] == (k == j) for k in range(len(self.vecs)))


def run(basis, cols, targets, m):
    """Columns in order: pivots (with combinations) and the representation
    of every non-pivot column; then each target's residual and solution."""
    out = []
    nb = 0
    for col in cols:
        x, comb = basis.reduce(col, np.zeros(m, np.uint8))
        p = lowest(x)
        if p >= 0:
            comb[nb] ^= 1
            basis.append(x, comb, p)
            out.append(("pivot", p, x.tobytes(), nb))
            nb += 1
        else:
            out.append(("rep", comb[:nb].tobytes()))
    for t in targets:
        x, comb = basis.reduce(t, np.zeros(m, np.uint8))
        out.append(("target", x.tobytes(), comb[:nb].tobytes() if not x.any() else None))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_reduced_echelon_equals_insertion_order(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 70))
    ncol = int(rng.integers(1, 2 * m + 3))
    dens = rng.uniform(0.02, 0.5)
    cols = [(rng.random(m) < dens).astype(np.uint8) for _ in range(ncol)]
    # targets: sums of random column subsets (in the span) and random vectors
    targets = []
    for _ in range(6):
        pick = rng.random(ncol) < 0.3
        t = np.zeros(m, np.uint8)
        for c, s in zip(cols, pick):
            if s:
                t ^= c
        targets.append(t)
        targets.append((rng.random(m) < 0.3).astype(np.uint8))
    a = run(Insertion(m), cols, targets, m)
    b = run(Reduced(m), cols, targets, m)
    assert a == b


def test_solution_reproduces_the_target():
    """The pivot combination of a target in the span sums the pivot columns
    to that target (checked on the reduced-echelon side)."""
    rng = np.random.default_rng(7)
    m = 40
    cols = [(rng.random(m) < 0.15).astype(np.uint8) for _ in range(30)]
    basis, pivcols, nb = Reduced(m), [], 0
    for col in cols:
        x, comb = basis.reduce(col, np.zeros(m, np.uint8))
        p = lowest(x)
        if p >= 0:
            comb[nb] ^= 1
            basis.append(x, comb, p)
            pivcols.append(col)
            nb += 1
    for _ in range(20):
        pick = rng.random(len(cols)) < 0.4
        t = np.zeros(m, np.uint8)
        for c, s in zip(cols, pick):
            if s:
                t ^= c
        x, comb = basis.reduce(t, np.zeros(m, np.uint8))
        assert not x.any()
        back = np.zeros(m, np.uint8)
        for i in np.flatnonzero(comb[:nb]):
            back ^= pivcols[i]
        assert np.array_equal(back, t)
