"""Python binding of libvibelsd (the MI355X VibeLSD decoder).

Argument marshalling only: every step of the decode path runs in the HIP
kernels of libvibelsd.so.  PyTorch provides device memory and the stream.
The C entry points keep their names here (vibe_graph_create, vibe_decode,
...); `Graph` wraps them for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvibelsd.so")

VIBE_OK, VIBE_EINVAL, VIBE_ENOMEM, VIBE_EHIP, VIBE_EUNSUPPORTED = 0, -1, -2, -3, -4
FLAG_BP_CONVERGED, FLAG_LSD_USED, FLAG_LSD_FAILED, FLAG_SATURATED = 1, 2, 4, 8
STATS_FIELDS = ("flags", "winner", "t_win", "n_conv", "lsd_clusters", "lsd_largest",
                "lsd_rounds", "member_iters")


class VibeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vibelsd error {code}: {msg}")
        self.code = code


class vibe_config(C.Structure):
    _fields_ = [("L", C.c_uint32), ("M", C.c_uint32), ("T_max", C.c_uint32),
                ("lsd_order", C.c_uint32), ("alpha", C.c_double), ("clamp", C.c_double),
                ("message_bits", C.c_uint32), ("schedule", C.c_uint32)]


class vibe_graph_info_t(C.Structure):
    _fields_ = [("m", C.c_uint32), ("n", C.c_uint32), ("k", C.c_uint32), ("L", C.c_uint32),
                ("M", C.c_uint32), ("T_max", C.c_uint32), ("nnz", C.c_uint64),
                ("max_row_degree", C.c_uint32), ("max_col_degree", C.c_uint32),
                ("levels_min", C.c_uint32), ("levels_max", C.c_uint32),
                ("chunks_min", C.c_uint32), ("chunks_max", C.c_uint32),
                ("message_bits", C.c_uint32), ("grad_width", C.c_uint32),
                ("device_bytes", C.c_uint64)]


class vibe_launch_t(C.Structure):
    _fields_ = [("slab_in_lds", C.c_int), ("grid", C.c_int), ("shots_per_wave", C.c_int),
                ("decisions_global", C.c_int), ("from_cache", C.c_int), ("ms", C.c_double)]


class vibe_request(C.Structure):
    _fields_ = [("graph", C.c_void_p), ("syndromes", C.c_void_p), ("B", C.c_uint64),
                ("corrections", C.c_void_p), ("observables", C.c_void_p), ("stats", C.c_void_p)]


class vibe_server_config(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("max_batch_requests", C.c_uint32), ("max_batch_shots", C.c_uint32),
                ("reserved", C.c_uint32), ("hbm_budget", C.c_uint64)]


_lib = None

EXPORTS = {
    "vibe_graph_create": (C.c_int, [C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(vibe_config), C.POINTER(C.c_void_p)]),
    "vibe_graph_destroy": (None, [C.c_void_p]),
    "vibe_graph_info": (C.c_int, [C.c_void_p, C.POINTER(vibe_graph_info_t)]),
    "vibe_decode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p]),
    "vibe_decode_packed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "vibe_decode_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "vibe_graph_get_schedules": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vibe_graph_set_alpha": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32]),
    "vibe_decode_plain": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "vibe_bp_ensemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_int,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vibe_lsd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "vibe_bp_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p,
                               C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vibe_grad_set_width": (C.c_int, [C.c_void_p, C.c_uint32]),
    "vibe_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "vibe_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "vibe_runtime_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "vibe_runtime_destroy": (None, [C.c_void_p]),
    "vibe_decode_ragged": (C.c_int, [C.c_void_p, C.POINTER(vibe_request), C.c_uint32, C.c_void_p]),
    "vibe_exec_create": (C.c_int, [C.POINTER(vibe_request), C.c_uint32, C.POINTER(C.c_void_p)]),
    "vibe_exec_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vibe_exec_destroy": (None, [C.c_void_p]),
    "vibe_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(vibe_launch_t)]),
    "vibe_set_launch": (C.c_int, [C.c_void_p, C.POINTER(vibe_launch_t)]),
    "vibe_get_launch": (C.c_int, [C.c_void_p, C.POINTER(vibe_launch_t)]),
    "vibe_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_uint32, C.POINTER(vibe_server_config),
                                     C.POINTER(C.c_void_p)]),
    "vibe_server_submit": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_uint64)]),
    "vibe_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]),
    "vibe_server_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                   C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "vibe_server_destroy": (None, [C.c_void_p]),
    "vibe_measure_slab_stream": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_void_p]),
    "vibe_last_error": (C.c_char_p, []),
    "vibe_version": (C.c_char_p, []),
}


def lib():
    """Load libvibelsd.so; there is no fallback if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_2508_15743_amd/_build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != VIBE_OK:
        raise VibeError(rc, lib().vibe_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def vibe_version() -> str:
    return lib().vibe_version().decode()


def vibe_graph_create(m, n, h_indptr, h_indices, priors, k, l_indptr, l_indices, perms, cfg):
    hp, hi, lp, li, pp = _u32(h_indptr), _u32(h_indices), _u32(l_indptr), _u32(l_indices), _u32(perms)
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().vibe_graph_create(m, n, hp.ctypes.data, hi.ctypes.data if hi.size else None,
                                   pr.ctypes.data, k, lp.ctypes.data, li.ctypes.data if li.size else None,
                                   pp.ctypes.data, C.byref(cfg), C.byref(out)))
    return out


def vibe_graph_destroy(handle):
    lib().vibe_graph_destroy(handle)


def vibe_graph_info(handle) -> dict:
    info = vibe_graph_info_t()
    _check(lib().vibe_graph_info(handle, C.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def vibe_decode(handle, syndromes, B, corrections, observables, stats, stream):
    _check(lib().vibe_decode(handle, _ptr(syndromes), B, _ptr(corrections), _ptr(observables),
                             _ptr(stats), stream))


def vibe_decode_packed(handle, words, B, corrections, observables, stats, stream):
    _check(lib().vibe_decode_packed(handle, _ptr(words), B, _ptr(corrections), _ptr(observables),
                                    _ptr(stats), stream))


def vibe_graph_set_alpha(handle, alpha):
    a = np.ascontiguousarray(alpha if alpha is not None else [], dtype=np.float64)
    _check(lib().vibe_graph_set_alpha(handle, a.ctypes.data if a.size else None, a.size))


def vibe_graph_get_schedules(handle, L, length) -> np.ndarray:
    out = np.zeros((L, length), dtype=np.uint32)
    _check(lib().vibe_graph_get_schedules(handle, out.ctypes.data))
    return out


def vibe_decode_noalloc(handle, syndromes, B, corrections, observables, stats, stream):
    _check(lib().vibe_decode_noalloc(handle, _ptr(syndromes), B, _ptr(corrections), _ptr(observables),
                                     _ptr(stats), stream))


def vibe_decode_plain(handle, syndromes, B, corrections, observables, stats, stream):
    _check(lib().vibe_decode_plain(handle, _ptr(syndromes), B, _ptr(corrections), _ptr(observables),
                                   _ptr(stats), stream))


def vibe_bp_ensemble(handle, syndromes, B, T_run, stop, t_conv, posteriors, ehat, stream):
    _check(lib().vibe_bp_ensemble(handle, _ptr(syndromes), B, T_run, 1 if stop else 0, _ptr(t_conv),
                                  _ptr(posteriors), _ptr(ehat), stream))


def vibe_lsd(handle, syndromes, soft, B, corrections, stats, stream):
    _check(lib().vibe_lsd(handle, _ptr(syndromes), _ptr(soft), B, _ptr(corrections), _ptr(stats),
                          stream))


def vibe_bp_grad(handle, syndromes, B, K, lam, alpha, eps, loss, dlam, dalpha, stream):
    _check(lib().vibe_bp_grad(handle, _ptr(syndromes), B, K, _ptr(lam), _ptr(alpha), eps, _ptr(loss),
                              _ptr(dlam), _ptr(dalpha), stream))


def vibe_runtime_create():
    out = C.c_void_p()
    _check(lib().vibe_runtime_create(C.byref(out)))
    return out


def vibe_runtime_destroy(rt):
    lib().vibe_runtime_destroy(rt)


def _requests(reqs):
    """[(Graph, syndromes, corrections, observables, stats or None)] -> ctypes array"""
    arr = (vibe_request * len(reqs))()
    for i, (G, s, c, o, st) in enumerate(reqs):
        arr[i] = vibe_request(G.handle, s.data_ptr(), s.shape[0], c.data_ptr(), o.data_ptr(),
                              st.data_ptr() if st is not None else None)
    return arr


def vibe_decode_ragged(rt, reqs, stream):
    arr = _requests(reqs)
    _check(lib().vibe_decode_ragged(rt, arr, len(reqs), stream))


def vibe_exec_create(reqs):
    arr = _requests(reqs)
    out = C.c_void_p()
    _check(lib().vibe_exec_create(arr, len(reqs), C.byref(out)))
    return out


def vibe_exec_launch(ex, stream):
    _check(lib().vibe_exec_launch(ex, stream))


def vibe_exec_destroy(ex):
    lib().vibe_exec_destroy(ex)


def _launch_dict(s):
    return {"slab_in_lds": s.slab_in_lds, "grid": s.grid, "shots_per_wave": s.shots_per_wave,
            "decisions_global": s.decisions_global, "from_cache": bool(s.from_cache), "ms": s.ms}


def vibe_autotune(handle, syndromes, B, stream):
    s = vibe_launch_t()
    _check(lib().vibe_autotune(handle, _ptr(syndromes), B, stream, C.byref(s)))
    return _launch_dict(s)


def vibe_set_launch(handle, slab_in_lds=0, grid=0, shots_per_wave=1, decisions_global=-1):
    s = vibe_launch_t(int(slab_in_lds), int(grid), int(shots_per_wave), int(decisions_global), 0, 0.0)
    _check(lib().vibe_set_launch(handle, C.byref(s)))


def vibe_get_launch(handle):
    s = vibe_launch_t()
    _check(lib().vibe_get_launch(handle, C.byref(s)))
    return _launch_dict(s)


def vibe_profile_enable(handle, enable):
    _check(lib().vibe_profile_enable(handle, 1 if enable else 0))


def vibe_profile_read(handle):
    ms = (C.c_double * 3)()
    n = (C.c_uint64 * 3)()
    _check(lib().vibe_profile_read(handle, ms, n))
    names = ("bp_ensemble", "select", "lsd")
    return {names[i]: (ms[i], n[i]) for i in range(3)}


def unpack_bits(words, n: int) -> np.ndarray:
    """[..., ceil(n/64)] int64 words (any device) -> [..., n] uint8 bits."""
    w = words.detach().cpu().numpy() if hasattr(words, "detach") else np.asarray(words)
    w = np.ascontiguousarray(w).view(np.uint64)
    b = np.unpackbits(w.view(np.uint8).reshape(*w.shape[:-1], 8 * w.shape[-1]), axis=-1, bitorder="little")
    return b[..., :n]


class Graph:
    """A detector error model resident on the current GPU, with its member
    schedules.  `perms` is [L, n]: the serial schedules of the members.
    message_bits=64 runs BP in FP64 (verification); 32 is the production
    setting.  schedule="parallel" runs every member with the flooding
    schedule (L=1, M=1 is the BP+LSD-0 baseline); schedule="layered" runs
    the check-serial schedule, and `perms` is then [L, m], one order of the
    checks per member."""

    def __init__(self, h_indptr, h_indices, priors, l_indptr, l_indices, perms, m=None, n=None,
                 L=32, M=5, T_max=20, alpha=0.625, clamp=1e6, lsd_order=0, message_bits=32,
                 schedule="serial"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libvibelsd needs a ROCm GPU (torch.cuda is not available)")
        lib()
        h_indptr = _u32(h_indptr)
        self.m = len(h_indptr) - 1 if m is None else m
        self.n = int(len(priors)) if n is None else n
        self.k = len(l_indptr) - 1
        self.L, self.M, self.T_max = L, M, T_max
        self.words = (self.n + 63) // 64
        self.message_bits = message_bits
        codes = {"serial": 0, "parallel": 1, "layered": 2}
        if schedule not in codes:
            raise ValueError("schedule must be 'serial', 'parallel' or 'layered'")
        self.schedule = schedule
        self.cfg = vibe_config(L, M, T_max, lsd_order, alpha, clamp, message_bits, codes[schedule])
        self.handle = vibe_graph_create(self.m, self.n, h_indptr, h_indices, priors, self.k,
                                        l_indptr, l_indices, perms, self.cfg)

    @classmethod
    def from_dem(cls, dem, perms, **cfg):
        return cls(dem.h_indptr, dem.h_indices, dem.priors, dem.l_indptr, dem.l_indices, perms,
                   m=dem.m, n=dem.n, **cfg)

    def info(self) -> dict:
        return vibe_graph_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            vibe_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _synd(self, syndromes):
        import torch
        if syndromes.dtype != torch.uint8 or syndromes.dim() != 2 or syndromes.shape[1] != self.m:
            raise ValueError(f"syndromes must be uint8 [B, {self.m}]")
        if not syndromes.is_cuda:
            raise ValueError("syndromes must be a device tensor")
        return syndromes.contiguous()

    def decode(self, syndromes, plain=False, with_stats=True, stream=None, out=None, noalloc=False):
        """-> (corrections int64 [B, words], observables uint8 [B, k], stats int32 [B, 8]).
        plain: one launch sequence per shot (vibe_decode_plain); noalloc: the
        library allocates nothing (vibe_decode_noalloc; pass `out` too for a
        call that allocates no device memory at all)."""
        import torch
        s = self._synd(syndromes)
        B = s.shape[0]
        dev = s.device
        if out is None:
            corr = torch.empty((B, self.words), dtype=torch.int64, device=dev)
            obs = torch.empty((B, max(self.k, 1)), dtype=torch.uint8, device=dev)
            st = torch.empty((B, 8), dtype=torch.int32, device=dev) if with_stats else None
        else:
            corr, obs, st = out
        fn = vibe_decode_plain if plain else (vibe_decode_noalloc if noalloc else vibe_decode)
        fn(self.handle, s, B, corr, obs, st, _stream(stream))
        return corr, obs, st

    def decode_packed(self, words, with_stats=True, stream=None):
        """Bit-packed syndromes int64 [B, ceil(m/64)] (check c in bit c % 64 of
        word c // 64) -> the results of decode()"""
        import torch
        wm = (self.m + 63) // 64
        if words.dtype != torch.int64 or words.dim() != 2 or words.shape[1] != wm or not words.is_cuda:
            raise ValueError(f"words must be an int64 device tensor [B, {wm}]")
        w = words.contiguous()
        B = w.shape[0]
        corr = torch.empty((B, self.words), dtype=torch.int64, device=w.device)
        obs = torch.empty((B, max(self.k, 1)), dtype=torch.uint8, device=w.device)
        st = torch.empty((B, 8), dtype=torch.int32, device=w.device) if with_stats else None
        vibe_decode_packed(self.handle, w, B, corr, obs, st, _stream(stream))
        return corr, obs, st

    def set_alpha(self, alpha=None):
        """One scaling factor per iteration (alpha_1 .. alpha_k; later
        iterations keep alpha_k); None returns to the constant alpha."""
        vibe_graph_set_alpha(self.handle, alpha)

    def schedules(self) -> np.ndarray:
        """The member schedules the graph holds: [L, n] (or [L, m] layered)."""
        return vibe_graph_get_schedules(self.handle, self.L, self.m if self.schedule == "layered" else self.n)

    def bp_ensemble(self, syndromes, T_run=None, stop=True, posteriors=True, ehat=True, stream=None):
        """-> (t_conv int32 [B, L], posteriors [B, L, n] (float32, or float64 when
        message_bits is 64) or None, ehat int64 [B, L, words] or None)"""
        import torch
        s = self._synd(syndromes)
        B = s.shape[0]
        dev = s.device
        T_run = self.T_max if T_run is None else T_run
        t = torch.empty((B, self.L), dtype=torch.int32, device=dev)
        pdt = torch.float64 if self.message_bits == 64 else torch.float32
        p = torch.empty((B, self.L, self.n), dtype=pdt, device=dev) if posteriors else None
        e = torch.empty((B, self.L, self.words), dtype=torch.int64, device=dev) if ehat else None
        vibe_bp_ensemble(self.handle, s, B, T_run, stop, t, p, e, _stream(stream))
        return t, p, e

    def lsd(self, syndromes, soft, stream=None):
        """-> (corrections int64 [B, words], stats int32 [B, 8])"""
        import torch
        s = self._synd(syndromes)
        B = s.shape[0]
        soft = soft.to(torch.float32).contiguous()
        if soft.shape != (B, self.n) or not soft.is_cuda:
            raise ValueError(f"soft must be a float32 device tensor [B, {self.n}]")
        corr = torch.empty((B, self.words), dtype=torch.int64, device=s.device)
        st = torch.empty((B, 8), dtype=torch.int32, device=s.device)
        vibe_lsd(self.handle, s, soft, B, corr, st, _stream(stream))
        return corr, st


def _graph_autotune(self, syndromes, stream=None):
    """Time the launch settings of decode() on these syndromes (or take them
    from the per-shape cache) and keep the fastest -> dict with slab_in_lds,
    grid, shots_per_wave, decisions_global, from_cache, ms."""
    return vibe_autotune(self.handle, self._synd(syndromes), syndromes.shape[0], _stream(stream))


def _graph_set_launch(self, slab_in_lds=0, grid=0, shots_per_wave=1, decisions_global=-1):
    """Apply launch settings (see vibe_set_launch)."""
    vibe_set_launch(self.handle, slab_in_lds, grid, shots_per_wave, decisions_global)


def _graph_get_launch(self):
    return vibe_get_launch(self.handle)


Graph.autotune = _graph_autotune
Graph.set_launch = _graph_set_launch
Graph.get_launch = _graph_get_launch


def _graph_bp_grad(self, syndromes, lam, alpha, eps=1e-7, stream=None):
    """Soft-syndrome loss of len(alpha) unrolled iterations of every member,
    summed over shots and members, and its gradient
    -> (loss [1], dlam [n], dalpha [K]), float64 device tensors.  lam and
    alpha are cast to the message precision (float32, or float64 when
    message_bits is 64)."""
    import torch
    s = self._synd(syndromes)
    dev = s.device
    pdt = torch.float64 if self.message_bits == 64 else torch.float32
    lam = lam.detach().to(device=dev, dtype=pdt).contiguous()
    alpha = alpha.detach().to(device=dev, dtype=pdt).contiguous()
    if lam.shape != (self.n,) or alpha.dim() != 1:
        raise ValueError(f"lam must have shape [{self.n}] and alpha one dimension")
    K = alpha.shape[0]
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    dlam = torch.empty(self.n, dtype=torch.float64, device=dev)
    dalpha = torch.empty(K, dtype=torch.float64, device=dev)
    vibe_bp_grad(self.handle, s, s.shape[0], K, lam, alpha, eps, loss, dlam, dalpha, _stream(stream))
    return loss, dlam, dalpha


Graph.bp_grad = _graph_bp_grad


def _graph_set_grad_width(self, width):
    """Chunk width of the gradient schedule (16, 32, 64; 0 = chosen per graph)."""
    _check(lib().vibe_grad_set_width(self.handle, width))


Graph.set_grad_width = _graph_set_grad_width


def _autograd_fn():
    import torch

    class BpLoss(torch.autograd.Function):
        """loss = BpLoss.apply(graph, syndromes, lam, alpha, eps): the loss
        and its gradient come from one vibe_bp_grad call; backward scales
        the stored gradient."""

        @staticmethod
        def forward(ctx, graph, syndromes, lam, alpha, eps=1e-7):
            loss, dlam, dalpha = graph.bp_grad(syndromes, lam, alpha, eps)
            ctx.save_for_backward(dlam.to(lam.dtype), dalpha.to(alpha.dtype))
            return loss[0].to(lam.dtype)

        @staticmethod
        def backward(ctx, g):
            dlam, dalpha = ctx.saved_tensors
            return None, None, g * dlam, g * dalpha, None

    return BpLoss


def bp_loss(graph, syndromes, lam, alpha, eps=1e-7):
    """Differentiable soft-syndrome loss of the unrolled ensemble (see
    Graph.bp_grad); gradients flow to lam and alpha."""
    global _BpLoss
    if _BpLoss is None:
        _BpLoss = _autograd_fn()
    return _BpLoss.apply(graph, syndromes, lam, alpha, eps)


_BpLoss = None


class Runtime:
    """Device workspace for ragged calls: decode() takes requests on several
    graphs and runs their BP ensembles as one persistent launch."""

    def __init__(self):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libvibelsd needs a ROCm GPU (torch.cuda is not available)")
        self.handle = vibe_runtime_create()

    @staticmethod
    def outputs(G, syndromes):
        import torch
        B, dev = syndromes.shape[0], syndromes.device
        return (torch.empty((B, G.words), dtype=torch.int64, device=dev),
                torch.empty((B, max(G.k, 1)), dtype=torch.uint8, device=dev),
                torch.empty((B, 8), dtype=torch.int32, device=dev))

    def decode(self, pairs, stream=None, outs=None):
        """pairs: [(Graph, syndromes uint8 [B, m])] -> [(corrections, observables, stats)]"""
        outs = outs or [self.outputs(G, s) for G, s in pairs]
        reqs = [(G, G._synd(s), c, o, st) for (G, s), (c, o, st) in zip(pairs, outs)]
        vibe_decode_ragged(self.handle, reqs, _stream(stream))
        return outs

    def close(self):
        if getattr(self, "handle", None):
            vibe_runtime_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Exec:
    """A captured ragged launch sequence over fixed buffers: refill the
    syndrome tensors, then launch()."""

    def __init__(self, pairs, outs=None):
        self.pairs = [(G, G._synd(s)) for G, s in pairs]
        self.outs = outs or [Runtime.outputs(G, s) for G, s in self.pairs]
        reqs = [(G, s, c, o, st) for (G, s), (c, o, st) in zip(self.pairs, self.outs)]
        self.handle = vibe_exec_create(reqs)

    def launch(self, stream=None):
        vibe_exec_launch(self.handle, _stream(stream))
        return self.outs

    def close(self):
        if getattr(self, "handle", None):
            vibe_exec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching over resident graphs, admission by HBM footprint
    (vibe_server_*).  submit() queues a request (device syndromes, ready when
    submitted) and returns a ticket at once; wait(ticket) blocks until it is
    decoded and returns its latency in ms.  Outputs are exactly those of
    Graph.decode on the request alone.  hbm_budget is the device pool in
    bytes (0: room for `slots` full batches)."""

    def __init__(self, graphs, slots=3, max_batch_requests=256, max_batch_shots=4096, hbm_budget=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libvibelsd needs a ROCm GPU (torch.cuda is not available)")
        self.graphs = list(graphs)
        arr = (C.c_void_p * len(self.graphs))(*[G.handle.value for G in self.graphs])
        cfg = vibe_server_config(slots, max_batch_requests, max_batch_shots, 0, hbm_budget)
        out = C.c_void_p()
        _check(lib().vibe_server_create(arr, len(self.graphs), C.byref(cfg), C.byref(out)))
        self.handle = out
        self._held = {}

    def submit(self, index, syndromes, out=None):
        """-> (ticket, (corrections, observables, stats))"""
        G = self.graphs[index]
        s = G._synd(syndromes)
        o = out or Runtime.outputs(G, s)
        t = C.c_uint64()
        _check(lib().vibe_server_submit(self.handle, index, _ptr(s), s.shape[0], _ptr(o[0]), _ptr(o[1]),
                                        _ptr(o[2]), C.byref(t)))
        self._held[t.value] = (s, o)
        return t.value, o

    def wait(self, ticket):
        ms = C.c_double()
        try:
            _check(lib().vibe_server_wait(self.handle, ticket, C.byref(ms)))
        finally:
            self._held.pop(ticket, None)
        return ms.value

    def info(self):
        b, r, pb, pk = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().vibe_server_info(self.handle, C.byref(b), C.byref(r), C.byref(pb), C.byref(pk)))
        return {"batches": b.value, "requests": r.value, "pool_bytes": pb.value, "peak_bytes": pk.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().vibe_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
