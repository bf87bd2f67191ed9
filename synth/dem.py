"""Detector error models (paper Sec. II.B): rows = detectors, columns = error
mechanisms with independent priors, plus a logical-observable matrix.

Three families, all on the triangular 6.6.6 colour code:
  * code capacity: H = face-vertex incidence, iid bit flips (one check type);
  * phenomenological: r noisy rounds of perfect-gate syndrome extraction with
    data flips (p) and measurement flips (q), then one perfect round;
  * circuit level: an X-memory experiment with one X and one Z ancilla per
    plaquette, a fixed CNOT order, and the "Uniform" noise of the paper's
    noise table (two-qubit depolarising after each CNOT, one-qubit
    depolarising on idle qubits, flips after resets and before measurements),
    all at the same rate p.

Everything here is input generation: no decoding arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .colour_code import SLOT_OFFSETS, triangular_666


@dataclass
class DEM:
    """A detector error model in CSR form (rows ascending, column indices
    ascending within a row)."""

    m: int
    n: int
    h_indptr: np.ndarray  # uint32, m + 1
    h_indices: np.ndarray  # uint32, nnz
    priors: np.ndarray  # float64, n
    k: int
    l_indptr: np.ndarray  # uint32, k + 1
    l_indices: np.ndarray  # uint32
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.h_indptr[-1])

    def dense_h(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        for c in range(self.m):
            h[c, self.h_indices[self.h_indptr[c]:self.h_indptr[c + 1]]] = 1
        return h

    def dense_l(self) -> np.ndarray:
        lo = np.zeros((self.k, self.n), dtype=np.uint8)
        for r in range(self.k):
            lo[r, self.l_indices[self.l_indptr[r]:self.l_indptr[r + 1]]] = 1
        return lo

    def column_lists(self):
        """cols[v] = ascending list of detectors of column v."""
        cols = [[] for _ in range(self.n)]
        for c in range(self.m):
            for v in self.h_indices[self.h_indptr[c]:self.h_indptr[c + 1]]:
                cols[int(v)].append(c)
        return cols

    def summary(self) -> dict:
        rowdeg = np.diff(self.h_indptr.astype(np.int64))
        coldeg = np.bincount(self.h_indices.astype(np.int64), minlength=self.n)
        return {
            "name": self.name,
            "m": self.m,
            "n": self.n,
            "nnz": self.nnz,
            "k": self.k,
            "max_row_degree": int(rowdeg.max()) if self.m else 0,
            "mean_row_degree": float(rowdeg.mean()) if self.m else 0.0,
            "max_col_degree": int(coldeg.max()) if self.n else 0,
            "mean_col_degree": float(coldeg.mean()) if self.n else 0.0,
            "sum_priors": float(self.priors.sum()),
        }


def csr_from_dense(a: np.ndarray):
    a = np.asarray(a, dtype=np.uint8)
    indptr = np.zeros(a.shape[0] + 1, dtype=np.uint32)
    idx = []
    for r in range(a.shape[0]):
        nz = np.flatnonzero(a[r])
        idx.append(nz)
        indptr[r + 1] = indptr[r] + len(nz)
    indices = np.concatenate(idx).astype(np.uint32) if idx else np.zeros(0, np.uint32)
    return indptr, indices


def dem_from_dense(h, priors, lobs, name="", meta=None) -> DEM:
    h = np.asarray(h, dtype=np.uint8)
    lobs = np.asarray(lobs, dtype=np.uint8)
    if lobs.ndim == 1:
        lobs = lobs[None, :]
    hp, hi = csr_from_dense(h)
    lp, li = csr_from_dense(lobs)
    return DEM(m=h.shape[0], n=h.shape[1], h_indptr=hp, h_indices=hi,
               priors=np.asarray(priors, dtype=np.float64).copy(),
               k=lobs.shape[0], l_indptr=lp, l_indices=li, name=name,
               meta=dict(meta or {}))


def dem_from_columns(m: int, k: int, col_dets, col_obs, priors, name="", meta=None) -> DEM:
    """Build a DEM from per-column detector lists and observable lists."""
    n = len(col_dets)
    rows = [[] for _ in range(m)]
    for v, dets in enumerate(col_dets):
        for c in dets:
            rows[c].append(v)
    lrows = [[] for _ in range(k)]
    for v, obs in enumerate(col_obs):
        for o in obs:
            lrows[o].append(v)

    def pack(rs):
        indptr = np.zeros(len(rs) + 1, dtype=np.uint32)
        for r, lst in enumerate(rs):
            indptr[r + 1] = indptr[r] + len(lst)
        indices = np.array([v for lst in rs for v in sorted(lst)], dtype=np.uint32)
        return indptr, indices

    hp, hi = pack(rows)
    lp, li = pack(lrows)
    return DEM(m=m, n=n, h_indptr=hp, h_indices=hi,
               priors=np.asarray(priors, dtype=np.float64), k=k,
               l_indptr=lp, l_indices=li, name=name, meta=dict(meta or {}))


# ---------------------------------------------------------------------------
# code capacity


def code_capacity_dem(d: int, p: float) -> DEM:
    """X flips on the data qubits, Z-type plaquette checks; the observable is
    the weight-n logical (all ones), which commutes with every plaquette."""
    code = triangular_666(d)
    h = code.check_matrix()
    lobs = np.ones((1, code.n), dtype=np.uint8)
    return dem_from_dense(h, np.full(code.n, p), lobs,
                          name=f"code_capacity_d{d}_p{p:g}",
                          meta={"d": d, "p": p, "family": "code_capacity"})


# ---------------------------------------------------------------------------
# phenomenological


def phenomenological_dem(d: int, rounds: int, p: float, q: float) -> DEM:
    """`rounds` noisy measurement rounds plus one perfect final round.

    Columns: a data-flip layer before each noisy round (rounds * n columns,
    layer-major), then a measurement flip for every (noisy round, check)
    (rounds * P columns).  Detector (c, r) = m_{c,r} xor m_{c,r-1} with
    m_{c,0} = 0, for r = 1 .. rounds + 1, round-major.
    """
    code = triangular_666(d)
    n, P = code.n, code.num_plaquettes
    qubit_checks = [[] for _ in range(n)]
    for c, members in enumerate(code.plaquettes):
        for qb, _ in members:
            qubit_checks[qb].append(c)
    m = P * (rounds + 1)
    col_dets, col_obs, pri = [], [], []
    for r in range(1, rounds + 1):  # data layer before round r
        for qb in range(n):
            col_dets.append(sorted(P * (r - 1) + c for c in qubit_checks[qb]))
            col_obs.append([0])
            pri.append(p)
    for r in range(1, rounds + 1):  # measurement flip in round r
        for c in range(P):
            col_dets.append([P * (r - 1) + c, P * r + c])
            col_obs.append([])
            pri.append(q)
    return dem_from_columns(m, 1, col_dets, col_obs, pri,
                            name=f"phenom_d{d}_r{rounds}_p{p:g}_q{q:g}",
                            meta={"d": d, "rounds": rounds, "p": p, "q": q,
                                  "family": "phenomenological"})


# ---------------------------------------------------------------------------
# circuit level


def _combine(p_old: float, p_new: float) -> float:
    # two independent mechanisms with the same signature act as one whose
    # probability is that of an odd number of them firing
    return p_old * (1.0 - p_new) + p_new * (1.0 - p_old)


def circuit_dem(d: int, rounds: int, p: float, return_stats: bool = False, noise: str = "uniform"):
    """X-memory circuit-level DEM at rate p.

    noise="uniform": every two-qubit gate is followed by two-qubit
    depolarising noise p, every idle qubit of a layer by one-qubit
    depolarising p, resets and readouts flip with probability p.
    noise="si1000" (Sec. IV.A's superconducting-inspired table): two-qubit
    gates p; idling in a gate layer p/10; idling in a readout or reset layer
    2p; resets flip with 2p and readouts with 5p.  The CNOT of this circuit is
    taken as the native two-qubit gate (the table's CZ), so no single-qubit
    Cliffords are added around it.

    Qubits: data 0..n-1, X ancillas n..n+P-1, Z ancillas n+P..n+2P-1.
    One round: reset the X ancillas in |+>; six CNOT layers ancilla->data
    (slot order of the plaquette offsets); read the X ancillas out and reset
    the Z ancillas in |0>; six CNOT layers data->ancilla; read the Z ancillas
    out.  Every qubit that no operation touches in a layer idles in it.  The data
    start in |+> (reset with the first round's ancillas) and end with an
    X-basis measurement.  Detectors, round-major with X before Z inside a
    round: X checks in rounds 1..R and a final one from the data readout; Z
    checks in rounds 2..R.  The observable is the product of all data X
    readouts.

    Error effects are found by propagating detector sensitivities backwards
    through the circuit: sx[q] / sz[q] is the set of detectors (bit mask,
    bit `m` = observable) flipped by an X / Z on qubit q at the current time.
    """
    if noise == "uniform":
        p_gate, p_idle_gate, p_idle_mr, p_reset, p_meas = p, p, p, p, p
    elif noise == "si1000":
        p_gate, p_idle_gate, p_idle_mr, p_reset, p_meas = p, p / 10, 2 * p, 2 * p, 5 * p
    else:
        raise ValueError(f"unknown noise model {noise!r}")
    code = triangular_666(d)
    n, P = code.n, code.num_plaquettes
    R = rounds
    xa = [n + c for c in range(P)]
    za = [n + P + c for c in range(P)]
    nq = n + 2 * P

    # detector indexing
    det_x = {}
    det_z = {}
    idx = 0
    for r in range(1, R + 2):
        for c in range(P):
            det_x[(c, r)] = idx
            idx += 1
        if 2 <= r <= R:
            for c in range(P):
                det_z[(c, r)] = idx
                idx += 1
    m = idx
    obs_bit = 1 << m

    def dets_mx(c, r):  # X-ancilla readout of plaquette c in round r
        return (1 << det_x[(c, r)]) | (1 << det_x[(c, r + 1)])

    def dets_mz(c, r):
        s = 0
        if r >= 2:
            s |= 1 << det_z[(c, r)]
        if r + 1 <= R:
            s |= 1 << det_z[(c, r + 1)]
        return s

    qubit_plaqs = [[] for _ in range(n)]
    for c, members in enumerate(code.plaquettes):
        for qb, _ in members:
            qubit_plaqs[qb].append(c)

    def dets_mfinal(qb):
        s = obs_bit
        for c in qubit_plaqs[qb]:
            s |= 1 << det_x[(c, R + 1)]
        return s

    # CNOT layers: list of (control, target) per layer
    x_layers, z_layers = [], []
    for slot in range(len(SLOT_OFFSETS)):
        xl, zl = [], []
        for c, members in enumerate(code.plaquettes):
            for qb, s in members:
                if s == slot:
                    xl.append((xa[c], qb))
                    zl.append((qb, za[c]))
        x_layers.append(xl)
        z_layers.append(zl)

    sx = [0] * nq
    sz = [0] * nq
    sigs: dict[int, float] = {}
    n_faults = 0

    def add(effect: int, prob: float):
        nonlocal n_faults
        n_faults += 1
        if effect == 0:
            return
        old = sigs.get(effect)
        sigs[effect] = prob if old is None else _combine(old, prob)

    def depol1(q, pr):
        a, b = sx[q], sz[q]
        add(a, pr / 3)
        add(a ^ b, pr / 3)
        add(b, pr / 3)

    def depol2(q1, q2, pr):
        e1 = (0, sx[q1], sx[q1] ^ sz[q1], sz[q1])
        e2 = (0, sx[q2], sx[q2] ^ sz[q2], sz[q2])
        for i in range(4):
            for j in range(4):
                if i or j:
                    add(e1[i] ^ e2[j], pr / 15)

    # --- final data readout (X basis): Z flip before it, then the readout
    for qb in range(n):
        sz[qb] = dets_mfinal(qb)
        sx[qb] = 0
    for qb in range(n):
        add(sz[qb], p_meas)  # readout flip

    all_q = list(range(nq))

    def cnot_layers_backward(layers):
        for layer in reversed(layers):
            busy = set()
            for (ctl, tgt) in layer:
                depol2(ctl, tgt, p_gate)
                busy.add(ctl)
                busy.add(tgt)
            for q in all_q:
                if q not in busy:
                    depol1(q, p_idle_gate)  # idle in this layer
            for (ctl, tgt) in layer:
                # backward through CNOT: X_ctl -> X_ctl X_tgt, Z_tgt -> Z_ctl Z_tgt
                sx[ctl] ^= sx[tgt]
                sz[tgt] ^= sz[ctl]

    for r in range(R, 0, -1):
        # layer: Z-ancilla readout (flip before it); data idle
        for c in range(P):
            sx[za[c]] = dets_mz(c, r)
            sz[za[c]] = 0
        for c in range(P):
            add(sx[za[c]], p_meas)
        for qb in range(n):
            depol1(qb, p_idle_mr)
        cnot_layers_backward(z_layers)
        # layer: X-ancilla readout (flip before it) and Z-ancilla reset (flip
        # after it); data idle
        for c in range(P):
            add(sx[za[c]], p_reset)
            sx[za[c]] = sz[za[c]] = 0
        for c in range(P):
            sz[xa[c]] = dets_mx(c, r)
            sx[xa[c]] = 0
        for c in range(P):
            add(sz[xa[c]], p_meas)
        for qb in range(n):
            depol1(qb, p_idle_mr)
        cnot_layers_backward(x_layers)
        # layer: X-ancilla reset (flip after it); data reset in round 1,
        # otherwise idle
        for c in range(P):
            add(sz[xa[c]], p_reset)
            sx[xa[c]] = sz[xa[c]] = 0
        if r == 1:
            for qb in range(n):
                add(sz[qb], p_reset)  # data prepared in |+> with a phase flip
                sx[qb] = sz[qb] = 0
        else:
            for qb in range(n):
                depol1(qb, p_idle_mr)

    det_mask = obs_bit - 1
    undetectable = [s for s in sigs if (s & det_mask) == 0]
    if undetectable:
        raise RuntimeError(f"{len(undetectable)} fault signatures flip only the observable")
    col_dets, col_obs, pri = [], [], []
    for s in sorted(sigs.keys()):
        dets = []
        x = s & det_mask
        while x:
            low = x & (-x)
            dets.append(low.bit_length() - 1)
            x ^= low
        col_dets.append(dets)
        col_obs.append([0] if s & obs_bit else [])
        pri.append(sigs[s])
    suffix = "" if noise == "uniform" else f"_{noise}"
    dem = dem_from_columns(m, 1, col_dets, col_obs, pri,
                           name=f"circuit_d{d}_r{R}_p{p:g}{suffix}",
                           meta={"d": d, "rounds": R, "p": p, "family": f"circuit_{noise}",
                                 "elementary_faults": n_faults})
    if return_stats:
        return dem, {"elementary_faults": n_faults, "signatures": len(sigs)}
    return dem
