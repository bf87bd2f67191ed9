"""Writes the oracle's per-shot results for the benchmark workloads to
tests/golden/, so that GPU tests can compare tens of thousands of shots
shot by shot without running the oracle for hours in the test run.

TEST INFRASTRUCTURE ONLY.  Calls the FP64 oracle (vibelsd_oracle.c through
oracle.py) on inputs from synth/ and nothing else.

Workloads (the decoder settings of the workload list):
  circuit_d9   circuit-level colour code d = 9, 9 rounds, Uniform p = 1e-3;
               L = 32, M = 5, T = 20, alpha = 0.625, LSD-0; permutations
               seed 2025, the first `shots` of the 32768-shot batch of seed
               2026 (the benchmark's inputs)
  phenom_d11   phenomenological colour code d = 11, 11 noisy rounds and a
               perfect one, p = q = 0.01; L = 32, M = 5, T = 50, alpha =
               0.625, LSD order 10; permutations seed 2030, 10^5 shots of
               seed 2031

Per shot it stores a digest of the correction (and, for the circuit
workload, its set bits), the observables, the flags, the winning member,
the LSD statistics and the tie witnesses: the smallest |L_v| of any decision
any member took, the smallest gap between soft values of any LSD rank
decision, and the weight gap between the chosen candidate and the next.

Usage: python -m oracle.fixtures circuit_d9 [--first F --count C] --threads 6
decodes shots [F, F + C) into a part file (progress is saved every chunk and
resumed from); python -m oracle.fixtures circuit_d9 --merge joins the parts
into tests/golden/oracle_circuit_d9.npz.  Parts may be computed on
different machines; overlapping shots must agree.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GOLDEN = os.path.join(ROOT, "tests", "golden")

WORKLOADS = {
    "circuit_d9": dict(kind="circuit", d=9, rounds=9, p=1e-3, L=32, M=5, T=20, alpha=0.625, lsd_order=0,
                       perm_seed=2025, sample_seed=2026, batch=32768, shots=20000, indices=True),
    "phenom_d11": dict(kind="phenom", d=11, rounds=11, p=0.01, q=0.01, L=32, M=5, T=50, alpha=0.625,
                       lsd_order=10, perm_seed=2030, sample_seed=2031, batch=100000, shots=100000,
                       indices=False),
}


def ehat_digest(ehat: np.ndarray) -> np.ndarray:
    """64-bit digest of each row of a 0/1 matrix [B, n] (blake2b of the
    little-endian bit-packed row), as uint64."""
    e = np.ascontiguousarray(np.atleast_2d(ehat), dtype=np.uint8)
    packed = np.packbits(e, axis=1, bitorder="little")
    out = np.empty(e.shape[0], np.uint64)
    for i in range(e.shape[0]):
        out[i] = int.from_bytes(hashlib.blake2b(packed[i].tobytes(), digest_size=8).digest(), "little")
    return out


def array_digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.tobytes() + str(a.dtype).encode() + str(a.shape).encode()).hexdigest()[:32]


def workload_inputs(name: str, shots: int | None = None):
    """(dem, perms, batch, spec) of a workload; the batch holds the first
    `shots` shots of the workload's full batch."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from synth.dem import circuit_dem, phenomenological_dem
    from synth.sample import permutations, sample

    w = WORKLOADS[name]
    if w["kind"] == "circuit":
        dem = circuit_dem(w["d"], w["rounds"], w["p"])
    else:
        dem = phenomenological_dem(w["d"], w["rounds"], w["p"], w["q"])
    perms = permutations(dem.n, w["L"], w["perm_seed"])
    b = sample(dem, w["batch"], w["sample_seed"])
    n = w["shots"] if shots is None else shots
    return dem, perms, b, n


def path_for(name: str) -> str:
    return os.path.join(GOLDEN, f"oracle_{name}.npz")


def part_path(name: str, first: int, count: int) -> str:
    return os.path.join(GOLDEN, f"oracle_{name}.shots_{first}_{first + count}.npz")


FIELDS = ("digest", "weight", "obs", "rec", "idx_len", "idx")


def run_part(name: str, first: int, count: int, threads: int, chunk: int) -> str:
    """Decode shots [first, first + count) of a workload with the oracle and
    store the raw per-shot results as a part file (progress is saved after
    every chunk and resumed from)."""
    from oracle import oracle as O

    w = WORKLOADS[name]
    dem, perms, b, _ = workload_inputs(name)
    g = O.OracleGraph(dem)
    dst = part_path(name, first, count)
    part = dst + ".partial.npz"
    done = 0
    acc = {k: [] for k in FIELDS}
    if os.path.exists(part):
        z = np.load(part)
        if int(z["n_target"]) == count and int(z["first"]) == first:
            done = int(z["done"])
            acc = {k: [z[k]] for k in FIELDS}
            print(f"{name}: resuming at {first + done}", flush=True)
    t0 = time.time()
    while done < count:
        lo, hi = first + done, first + min(count, done + chunk)
        r = O.decode(g, perms, b.syndromes[lo:hi], L=w["L"], M=w["M"], T=w["T"], alpha=w["alpha"],
                     threads=threads, lsd_order=w["lsd_order"])
        e = r["ehat"]
        nz = [np.flatnonzero(row).astype(np.uint32) for row in e]
        for k, v in (("digest", ehat_digest(e)), ("weight", e.sum(1).astype(np.uint32)), ("obs", r["obs"]),
                     ("rec", r["rec"]), ("idx_len", np.array([len(x) for x in nz], np.uint32)),
                     ("idx", np.concatenate(nz) if nz else np.zeros(0, np.uint32))):
            acc[k].append(v)
        done = hi - first
        acc = {k: [np.concatenate(v)] for k, v in acc.items()}
        np.savez(part, n_target=count, first=first, done=done, **{k: v[0] for k, v in acc.items()})
        print(f"{name}: shots {first}..{hi} of {first}..{first + count} done, {time.time() - t0:.0f} s", flush=True)
    np.savez(dst, first=first, count=count, **{k: v[0] for k, v in acc.items()})
    os.remove(part)
    return dst


def _parts(name: str):
    """(first, count, arrays) of every stored part and unfinished run."""
    import glob

    out = []
    for f in sorted(glob.glob(os.path.join(GOLDEN, f"oracle_{name}.shots_*.npz*"))):
        z = np.load(f)
        first = int(z["first"]) if "first" in z.files else 0
        count = int(z["done"]) if "done" in z.files else int(z["count"])
        out.append((first, count, {k: z[k] for k in FIELDS}))
    return out


def merge(name: str, shots: int | None = None) -> str:
    """Join the parts of a workload into its fixture (shots [0, n)), written
    to tests/golden; where parts overlap, their shots must agree."""
    w = WORKLOADS[name]
    dem, perms, b, n = workload_inputs(name, shots)
    digest = np.zeros(n, np.uint64)
    have = np.zeros(n, bool)
    rows = [None] * n
    for first, count, z in _parts(name):
        ends = np.concatenate(([0], np.cumsum(z["idx_len"]))).astype(np.int64)
        for j in range(min(count, n - first) if first < n else 0):
            i = first + j
            row = (z["digest"][j], z["weight"][j], z["obs"][j], z["rec"][j], z["idx"][ends[j]:ends[j + 1]])
            if have[i]:
                assert row[0] == digest[i] and np.array_equal(row[3], rows[i][3], equal_nan=True), (name, i)
                continue
            have[i], digest[i], rows[i] = True, row[0], row
    missing = np.flatnonzero(~have)
    if len(missing):
        raise SystemExit(f"{name}: {len(missing)} shots have no result yet (first {missing[0]})")
    rec = np.stack([r[3] for r in rows])
    meta = dict(w, workload=dem.name, m=dem.m, n=dem.n, nnz=dem.nnz, shots=n,
                syndromes_sha=array_digest(b.syndromes[:n]), perms_sha=array_digest(perms),
                observables_sha=array_digest(b.observables[:n]))
    out = dict(
        meta=np.array(json.dumps(meta)),
        ehat_digest=digest,
        ehat_weight=np.array([r[1] for r in rows], np.uint32),
        obs=np.stack([r[2] for r in rows]).astype(np.uint8),
        flags=rec[:, 0].astype(np.uint8),
        winner=rec[:, 1].astype(np.int16),
        t_win=rec[:, 2].astype(np.uint8),
        lsd_clusters=rec[:, 4].astype(np.uint32),
        lsd_largest=rec[:, 5].astype(np.uint32),
        lsd_rounds=rec[:, 6].astype(np.uint32),
        min_abs_post=rec[:, 7],
        min_q_gap=rec[:, 8],
        w_gap=rec[:, 10],
    )
    if w["indices"]:
        lens = np.array([len(r[4]) for r in rows], np.uint32)
        out["ehat_indptr"] = np.concatenate(([0], np.cumsum(lens))).astype(np.uint32)
        out["ehat_indices"] = np.concatenate([r[4] for r in rows]).astype(np.uint16 if dem.n < 65536 else np.uint32)
    dst = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.npz")
    np.savez_compressed(dst, **out)
    print(f"{name}: wrote {dst} ({os.path.getsize(dst)} bytes, {n} shots)", flush=True)
    return dst


def load(name: str) -> dict:
    """The stored results of a workload (plain arrays; meta as a dict)."""
    z = np.load(path_for(name))
    out = {k: z[k] for k in z.files}
    out["meta"] = json.loads(str(out["meta"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--first", type=int, default=0, help="first shot of the part to decode")
    ap.add_argument("--count", type=int, default=None, help="shots of the part (default: the workload's)")
    ap.add_argument("--threads", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--chunk", type=int, default=240)
    ap.add_argument("--merge", action="store_true", help="join the stored parts into the fixture")
    ap.add_argument("--dir", default=None, help="where parts are written and read (default tests/golden)")
    a = ap.parse_args()
    global GOLDEN
    if a.dir:
        GOLDEN = a.dir
        os.makedirs(GOLDEN, exist_ok=True)
    if a.merge:
        merge(a.workload, a.count)
        return
    count = a.count if a.count is not None else WORKLOADS[a.workload]["shots"] - a.first
    run_part(a.workload, a.first, count, a.threads, a.chunk)


if __name__ == "__main__":
    main()
