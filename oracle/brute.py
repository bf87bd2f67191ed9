"""Brute-force references used to pin the oracle (numpy, tiny inputs only).

TEST INFRASTRUCTURE ONLY.  Nothing here calls the oracle or the HIP path.

  * ml_coset_table: exact maximum-likelihood coset decoding by enumerating
    every error (the decoding objective of paper Sec. II.B);
  * min_weight_marginals: W_b(v) = min { W(e) : H e = s, e_v = b } with
    W(e) = sum_v e_v ln((1 - p_v) / p_v), by enumeration;
  * gf2_rank / gf2_in_span / greedy_basis / solve_on: dense GF(2) linear
    algebra written independently of the oracle's elimination.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_errors(n: int) -> np.ndarray:
    """Every length-n binary vector, shape [2**n, n], uint8."""
    idx = np.arange(1 << n, dtype=np.int64)
    return ((idx[:, None] >> np.arange(n)) & 1).astype(np.uint8)


def ml_coset_table(H, Lobs, priors):
    """For every syndrome reachable, the most likely observable class.

    Returns (table: dict syndrome-bytes -> observable tuple, ler_poly) where
    ler_poly is the exact ML logical failure probability at these priors.
    """
    H = np.asarray(H, np.int64)
    Lobs = np.atleast_2d(np.asarray(Lobs, np.int64))
    p = np.asarray(priors, np.float64)
    n = H.shape[1]
    E = all_errors(n).astype(np.int64)
    prob = np.prod(np.where(E == 1, p, 1 - p), axis=1)
    S = E @ H.T % 2
    O = E @ Lobs.T % 2
    mass = {}
    for s, o, w in zip(map(bytes, S.astype(np.uint8)), map(tuple, O), prob):
        mass.setdefault(s, {}).setdefault(o, 0.0)
        mass[s][o] += w
    table = {}
    fail = 0.0
    for s, cls in mass.items():
        best = max(cls.items(), key=lambda kv: kv[1])
        table[s] = best[0]
        fail += sum(cls.values()) - best[1]
    return table, fail


def min_weight_marginals(H, lam, s):
    """[n, 2] array of W_b(v); +inf where no solution with e_v = b exists."""
    H = np.asarray(H, np.int64)
    n = H.shape[1]
    E = all_errors(n).astype(np.int64)
    ok = np.all(E @ H.T % 2 == np.asarray(s, np.int64)[None, :], axis=1)
    W = E @ np.asarray(lam, np.float64)
    out = np.full((n, 2), np.inf)
    for b in (0, 1):
        for v in range(n):
            sel = ok & (E[:, v] == b)
            if sel.any():
                out[v, b] = W[sel].min()
    return out


def gf2_rank(A) -> int:
    A = (np.asarray(A, np.uint8) & 1).copy()
    rows, cols = A.shape
    r = 0
    for j in range(cols):
        nz = np.flatnonzero(A[r:, j])
        if len(nz) == 0:
            continue
        i = r + nz[0]
        A[[r, i]] = A[[i, r]]
        hit = np.flatnonzero(A[:, j])
        hit = hit[hit != r]
        A[hit] ^= A[r]
        r += 1
        if r == rows:
            break
    return r


def gf2_in_span(A, b) -> bool:
    A = np.asarray(A, np.uint8)
    if A.shape[1] == 0:
        return not np.any(b)
    return gf2_rank(A) == gf2_rank(np.column_stack([A, np.asarray(b, np.uint8)]))


def greedy_basis(A, order):
    """Columns of A taken in `order`; keep a column iff it raises the rank."""
    kept = []
    for j in order:
        trial = kept + [j]
        if gf2_rank(A[:, trial]) == len(trial):
            kept.append(j)
    return kept


def solve_on(A, cols, b):
    """The unique x supported on `cols` (independent) with A x = b, by
    enumeration over the 2**len(cols) supports (len(cols) <= 20)."""
    A = np.asarray(A, np.int64)
    b = np.asarray(b, np.int64)
    for bits in itertools.product((0, 1), repeat=len(cols)):
        x = np.zeros(A.shape[1], np.int64)
        x[list(cols)] = bits
        if np.array_equal(A @ x % 2, b % 2):
            return x.astype(np.uint8)
    return None
