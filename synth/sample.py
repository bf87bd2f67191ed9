"""Seeded sampling of syndromes from a detector error model, plus the seeded
schedule permutations.  Both sides of every comparison (the HIP path and the
oracle) receive their inputs from here; nothing in this module decodes.

Every column fires independently with its prior.  Per column the number of
firing shots is Binomial(shots, p); the firing shots are a uniform subset of
that size.  s = H e mod 2 and obs = Lobs e mod 2 per shot.  The generator is
numpy's Philox bit generator keyed by the seed, so a (dem, shots, seed) triple
always yields the same batch.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .dem import DEM


@dataclass
class Batch:
    syndromes: np.ndarray  # uint8 [shots, m]
    observables: np.ndarray  # uint8 [shots, k]
    err_shot: np.ndarray  # int64: shot index of every fired mechanism
    err_col: np.ndarray  # int64: column of every fired mechanism

    @property
    def shots(self) -> int:
        return self.syndromes.shape[0]

    def errors_dense(self, n: int) -> np.ndarray:
        e = np.zeros((self.shots, n), dtype=np.uint8)
        np.bitwise_xor.at(e, (self.err_shot, self.err_col), 1)
        return e


def _col_members(indptr, indices, n):
    """CSR rows -> per-column lists as (col_ptr, col_rows)."""
    indptr = indptr.astype(np.int64)
    rows = np.repeat(np.arange(len(indptr) - 1, dtype=np.int64), np.diff(indptr))
    cols = indices.astype(np.int64)
    order = np.argsort(cols, kind="stable")
    col_rows = rows[order]
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(col_ptr, cols + 1, 1)
    col_ptr = np.cumsum(col_ptr)
    return col_ptr, col_rows


def sample(dem: DEM, shots: int, seed: int) -> Batch:
    rng = np.random.Generator(np.random.Philox(key=seed))
    counts = rng.binomial(shots, dem.priors)
    err_shot = np.empty(int(counts.sum()), dtype=np.int64)
    err_col = np.repeat(np.arange(dem.n, dtype=np.int64), counts)
    pos = 0
    for v in np.flatnonzero(counts):
        k = int(counts[v])
        err_shot[pos:pos + k] = rng.choice(shots, size=k, replace=False)
        pos += k
    synd = _parity(dem.h_indptr, dem.h_indices, dem.n, dem.m, shots, err_shot, err_col)
    obs = _parity(dem.l_indptr, dem.l_indices, dem.n, dem.k, shots, err_shot, err_col)
    return Batch(syndromes=synd, observables=obs, err_shot=err_shot, err_col=err_col)


def _parity(indptr, indices, n, rows, shots, err_shot, err_col):
    col_ptr, col_rows = _col_members(indptr, indices, n)
    out = np.zeros((shots, rows), dtype=np.uint8)
    if len(err_col) == 0 or rows == 0:
        return out
    deg = col_ptr[err_col + 1] - col_ptr[err_col]
    sh = np.repeat(err_shot, deg)
    starts = np.repeat(col_ptr[err_col], deg)
    within = np.arange(len(sh), dtype=np.int64) - np.repeat(np.cumsum(deg) - deg, deg)
    rr = col_rows[starts + within]
    lin = sh * rows + rr
    lin.sort()
    # an index that occurs an odd number of times is a flipped row
    if len(lin):
        brk = np.flatnonzero(np.diff(lin)) + 1
        starts_run = np.concatenate(([0], brk))
        lens = np.diff(np.concatenate((starts_run, [len(lin)])))
        odd = lin[starts_run[lens % 2 == 1]]
        out.reshape(-1)[odd] = 1
    return out


def permutations(n: int, L: int, seed: int) -> np.ndarray:
    """L uniformly random permutations of range(n), uint32 [L, n]: the
    offline serial schedules of the ensemble members."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    return np.stack([rng.permutation(n) for _ in range(L)]).astype(np.uint32)


def syndromes_from_errors(dem: DEM, e: np.ndarray) -> np.ndarray:
    """s = H e mod 2 for a dense error batch (used for hand-made cases)."""
    e = np.atleast_2d(np.asarray(e, dtype=np.uint8))
    return (e.astype(np.int64) @ dem.dense_h().T.astype(np.int64) % 2).astype(np.uint8)
