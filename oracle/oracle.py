"""ctypes front end of the FP64 CPU oracle (vibelsd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library and its Python binding
never import this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vibelsd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
REC = 16  # doubles per shot record

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = C.CDLL(LIB)
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


I32, U8, U32, F64 = C.c_int32, C.c_uint8, C.c_uint32, C.c_double


def prior_llr(priors, lim: float = 1e6) -> np.ndarray:
    """Channel LLR of each column: ln((1 - p) / p), clamped to +-lim."""
    p = np.asarray(priors, dtype=np.float64)
    if np.any(p <= 0) or np.any(p >= 1):
        raise ValueError("priors must lie in (0, 1)")
    return np.clip(np.log((1.0 - p) / p), -lim, lim)


class OracleGraph:
    """CSR, CSC and the CSC->CSR edge map of a DEM, as int32 arrays."""

    def __init__(self, dem):
        self.m, self.n, self.k = dem.m, dem.n, dem.k
        self.rp = dem.h_indptr.astype(np.int32)
        self.ri = dem.h_indices.astype(np.int32)
        E = int(self.rp[-1])
        rows = np.repeat(np.arange(self.m, dtype=np.int32), np.diff(self.rp))
        order = np.lexsort((rows, self.ri))  # by column, then row
        self.ci = rows[order].astype(np.int32)
        self.ce = order.astype(np.int32)  # CSR position of each CSC entry
        cnt = np.bincount(self.ri, minlength=self.n)
        self.cp = np.zeros(self.n + 1, dtype=np.int32)
        self.cp[1:] = np.cumsum(cnt)
        self.lp = dem.l_indptr.astype(np.int32)
        self.li = dem.l_indices.astype(np.int32)
        self.priors = dem.priors.astype(np.float64)
        self.E = E

    def args(self):
        return (self.m, self.n, _p(self.rp, I32), _p(self.ri, I32), _p(self.cp, I32),
                _p(self.ci, I32), _p(self.ce, I32))


def bp(g: OracleGraph, s, perm=None, T=20, alpha=0.625, lim=1e6, stop=True, trace=False,
       lam=None):
    """One min-sum decoder (Algorithm 1).  perm=None -> parallel schedule."""
    L = lib()
    s = np.ascontiguousarray(s, dtype=np.uint8)
    lam = prior_llr(g.priors, lim) if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    al = np.full(T, alpha, dtype=np.float64) if np.ndim(alpha) == 0 else \
        np.ascontiguousarray(alpha, dtype=np.float64)
    tconv = C.c_int(0)
    iters = C.c_int(0)
    mn = C.c_double(0)
    ehat = np.zeros(g.n, np.uint8)
    post = np.zeros(g.n, np.float64)
    tr = np.full((T, g.n), np.nan) if trace else None
    pp = None
    if perm is not None:
        pp = np.ascontiguousarray(perm, dtype=np.uint32)
    rc = L.or_bp(*g.args(), _p(lam, F64), _p(s, U8), _p(pp, U32) if pp is not None else None,
                 C.c_int(T), _p(al, F64), C.c_double(lim), C.c_int(1 if stop else 0),
                 C.byref(tconv), _p(ehat, U8), _p(post, F64), C.byref(iters), C.byref(mn),
                 _p(tr, F64) if trace else None)
    if rc:
        raise MemoryError("oracle bp failed")
    return {"t_conv": tconv.value, "ehat": ehat, "post": post, "iters": iters.value,
            "min_abs_post": mn.value, "trace": tr}


def bp_layered(g: OracleGraph, s, cperm, T=20, alpha=0.625, lim=1e6, stop=True, trace=False, lam=None):
    """One min-sum decoder with the layered (check-serial) schedule: the
    checks in the order cperm (or_bp_layered).  Same outputs as bp()."""
    L = lib()
    s = np.ascontiguousarray(s, dtype=np.uint8)
    lam = prior_llr(g.priors, lim) if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    al = np.full(T, alpha, dtype=np.float64) if np.ndim(alpha) == 0 else \
        np.ascontiguousarray(alpha, dtype=np.float64)
    tconv, iters, mn = C.c_int(0), C.c_int(0), C.c_double(0)
    ehat = np.zeros(g.n, np.uint8)
    post = np.zeros(g.n, np.float64)
    tr = np.full((T, g.n), np.nan) if trace else None
    cp = np.ascontiguousarray(cperm, dtype=np.uint32)
    if cp.shape != (g.m,):
        raise ValueError("cperm must be a permutation of the m checks")
    rc = L.or_bp_layered(*g.args(), _p(lam, F64), _p(s, U8), _p(cp, U32), C.c_int(T), _p(al, F64),
                         C.c_double(lim), C.c_int(1 if stop else 0), C.byref(tconv), _p(ehat, U8),
                         _p(post, F64), C.byref(iters), C.byref(mn), _p(tr, F64) if trace else None)
    if rc:
        raise MemoryError("oracle bp failed")
    return {"t_conv": tconv.value, "ehat": ehat, "post": post, "iters": iters.value,
            "min_abs_post": mn.value, "trace": tr}


def bp_loss(g: OracleGraph, s, lam, alpha, K, perm=None, lim=1e6, eps=1e-7):
    """Soft-syndrome loss after K unrolled iterations (or_bp_loss):
    -> (loss, branch signature, final posteriors)."""
    L = lib()
    L.or_bp_loss.restype = C.c_double
    s = np.ascontiguousarray(s, dtype=np.uint8)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    al = np.ascontiguousarray(np.broadcast_to(alpha, (K,)), dtype=np.float64)
    pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.uint32)
    sig = C.c_uint64(0)
    post = np.zeros(g.n, np.float64)
    loss = L.or_bp_loss(*g.args(), _p(lam, F64), _p(s, U8), _p(pp, U32) if pp is not None else None,
                        C.c_int(K), _p(al, F64), C.c_double(lim), C.c_double(eps), C.byref(sig),
                        _p(post, F64))
    return loss, sig.value, post


def fd_grad(g: OracleGraph, s, lam, alpha, K, perm=None, h=1e-6, lim=1e6, eps=1e-7, idx=None):
    """Reference gradient of bp_loss by central differences in FP64, with
    respect to lam[v] (every v, or the v in idx; the others stay 0) and every
    alpha[t].  Each entry comes with a flag: True where the branch signature
    at +h and -h equals the one at the centre (the loss is smooth there, so
    the difference quotient is the derivative to O(h^2))."""
    lam = np.asarray(lam, dtype=np.float64)
    al = np.asarray(np.broadcast_to(alpha, (K,)), dtype=np.float64).copy()
    _, sig0, _ = bp_loss(g, s, lam, al, K, perm, lim, eps)
    dl, okl = np.zeros(g.n), np.zeros(g.n, bool)
    for v in (range(g.n) if idx is None else idx):
        lp, lm = lam.copy(), lam.copy()
        lp[v] += h
        lm[v] -= h
        fp, sp, _ = bp_loss(g, s, lp, al, K, perm, lim, eps)
        fm, sm, _ = bp_loss(g, s, lm, al, K, perm, lim, eps)
        dl[v] = (fp - fm) / (2 * h)
        okl[v] = sp == sig0 and sm == sig0
    da, oka = np.zeros(K), np.zeros(K, bool)
    for t in range(K):
        ap, am = al.copy(), al.copy()
        ap[t] += h
        am[t] -= h
        fp, sp, _ = bp_loss(g, s, lam, ap, K, perm, lim, eps)
        fm, sm, _ = bp_loss(g, s, lam, am, K, perm, lim, eps)
        da[t] = (fp - fm) / (2 * h)
        oka[t] = sp == sig0 and sm == sig0
    return dl, okl, da, oka


def lsd(g: OracleGraph, s, q, order=0, lim=1e6):
    """LSD on soft input q (lower = more likely flipped): LSD-0, or with
    order > 0 the combination sweep over each cluster's non-pivot columns,
    weighted by the prior LLRs."""
    L = lib()
    s = np.ascontiguousarray(s, dtype=np.uint8)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ehat = np.zeros(g.n, np.uint8)
    st = np.zeros(6, np.int32)
    gap = C.c_double(0)
    cl = np.zeros(g.m, np.int32)
    bl = np.zeros(g.n, np.int32)
    lam = prior_llr(g.priors, lim)
    rc = L.or_lsd(g.m, g.n, _p(g.rp, I32), _p(g.ri, I32), _p(g.cp, I32), _p(g.ci, I32),
                  _p(s, U8), _p(q, F64), C.c_int(order), _p(lam, F64), _p(ehat, U8), _p(st, I32), C.byref(gap),
                  _p(cl, I32), _p(bl, I32))
    return {"ehat": ehat, "failed": bool(rc), "clusters": int(st[0]), "largest": int(st[1]),
            "rounds": int(st[2]), "total_bits": int(st[4]), "min_gap": gap.value,
            "check_label": cl, "bit_label": bl}


def decode(g: OracleGraph, perms, synd, L=32, M=5, T=20, alpha=0.625, lim=1e6,
           schedule="serial", threads=None, want_members=False, want_q=False, lsd_order=0):
    """The full VibeLSD decoder over a batch of syndromes [B, m]."""
    lb = lib()
    synd = np.ascontiguousarray(synd, dtype=np.uint8)
    if synd.ndim == 1:
        synd = synd[None, :]
    B = synd.shape[0]
    perms = np.ascontiguousarray(perms, dtype=np.uint32)
    if schedule == "serial" and perms.shape != (L, g.n):
        raise ValueError("perms must be [L, n]")
    if schedule == "layered" and perms.shape != (L, g.m):
        raise ValueError("layered schedules take check permutations [L, m]")
    sched = {"serial": 0, "parallel": 1, "layered": 2}[schedule]
    lam = prior_llr(g.priors, lim)
    al = np.full(T, alpha, dtype=np.float64) if np.ndim(alpha) == 0 else \
        np.ascontiguousarray(alpha, dtype=np.float64)
    ehat = np.zeros((B, g.n), np.uint8)
    obs = np.zeros((B, g.k), np.uint8)
    rec = np.zeros((B, REC), np.float64)
    tm = np.zeros((B, L), np.int32) if want_members else None
    qo = np.full((B, g.n), np.nan) if want_q else None
    threads = threads or min(16, os.cpu_count() or 1)
    lb.or_decode_batch(g.m, g.n, g.k, _p(g.rp, I32), _p(g.ri, I32), _p(g.cp, I32),
                       _p(g.ci, I32), _p(g.ce, I32), _p(g.lp, I32), _p(g.li, I32),
                       _p(lam, F64), _p(perms, U32), C.c_int(L), C.c_int(M), C.c_int(T),
                       _p(al, F64), C.c_double(lim), C.c_int(sched), C.c_int(lsd_order),
                       _p(synd, U8), C.c_int64(B), C.c_int(threads), _p(ehat, U8), _p(obs, U8),
                       _p(rec, F64), _p(tm, I32) if tm is not None else None,
                       _p(qo, F64) if qo is not None else None)
    out = {"ehat": ehat, "obs": obs, "rec": rec,
           "converged": (rec[:, 0].astype(np.int64) & 1) == 1,
           "lsd_used": (rec[:, 0].astype(np.int64) & 2) == 2,
           "lsd_failed": (rec[:, 0].astype(np.int64) & 4) == 4,
           "saturated": (rec[:, 0].astype(np.int64) & 8) == 8,
           "winner": rec[:, 1].astype(np.int64), "t_win": rec[:, 2].astype(np.int64),
           "n_conv": rec[:, 3].astype(np.int64), "min_abs_post": rec[:, 7],
           "min_q_gap": rec[:, 8], "w_gap": rec[:, 10]}
    if tm is not None:
        out["t_members"] = tm
    if qo is not None:
        out["q"] = qo
    return out
