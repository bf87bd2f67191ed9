"""Ragged batching, captured launch sequences and autotuning (through the C ABI).

Every request of a ragged call must come out exactly as vibe_decode gives it
alone: same corrections, observables and deterministic stats fields.  Each
request's outputs from the ragged launch and from captured replays are also
compared with the FP64 oracle on a sample of its shots, to the FP32 bar of
test_gpu_parity.py (the oracle decodes each shot on its own with the graph's
schedules, so this checks the per-request results of Sec. III.D.2 directly,
not only their equality with another HIP path).
"""
import numpy as np
import pytest

from synth.dem import circuit_dem, code_capacity_dem, phenomenological_dem
from synth.sample import permutations, sample

from parity_helpers import check_valid, sampled_oracle_parity

pytestmark = pytest.mark.gpu

DET = [0, 1, 2, 4, 5, 6]  # stats fields that do not depend on timing


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15743_amd as P

    P.lib()
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _graphs(schedule="serial"):
    import paper_2508_15743_amd as P

    specs = [(code_capacity_dem(5, 0.05), 16, 5, 32), (circuit_dem(5, 5, 1e-3), 32, 5, 20),
             (phenomenological_dem(7, 7, 0.01, 0.01), 24, 5, 30), (circuit_dem(7, 7, 1e-3), 32, 5, 20)]
    out = []
    for i, (dem, L, M, T) in enumerate(specs):
        if schedule == "parallel":
            L, M = 1, 1
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 40 + i), L=L, M=M, T_max=T, schedule=schedule)
        out.append((dem, G))
    return out


def _check_same(torch, got, want):
    for (c1, o1, s1), (c2, o2, s2) in zip(got, want):
        assert torch.equal(c1, c2)
        assert torch.equal(o1, o2)
        assert torch.equal(s1[:, DET], s2[:, DET])


def _check_oracle(dems, pairs, outs, n_sample, seed, schedules=None):
    """Each request's ragged outputs against the oracle on a sample of its
    shots; corrections satisfy H e = s on every shot LSD did not flag."""
    import paper_2508_15743_amd as P

    for i, (dem, (G, s), (c, o, st)) in enumerate(zip(dems, pairs, outs)):
        synd = s.cpu().numpy()
        e, st = P.unpack_bits(c, dem.n), st.cpu().numpy()
        check_valid(dem, e, synd, st)
        sch = schedules[i] if schedules else "serial"
        print(sampled_oracle_parity(dem, G, synd, e, st, n_sample, seed + i, f"ragged request {i} {dem.name} {sch}",
                                    schedule=sch), flush=True)


@pytest.mark.parametrize("schedule", ["serial", "parallel"])
def test_ragged_equals_single(torch_cuda, schedule):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    gs = _graphs(schedule)
    sizes = [700, 1, 0, 333]  # an empty request and a single shot among them
    pairs = [(G, _dev(torch, sample(dem, B, 90 + i).syndromes) if B else
              torch.zeros((0, dem.m), dtype=torch.uint8, device="cuda:0"))
             for i, ((dem, G), B) in enumerate(zip(gs, sizes))]
    want = [G.decode(s) for G, s in pairs]
    rt = P.Runtime()
    got = rt.decode(pairs)
    _check_same(torch, got, want)
    _check_oracle([dem for dem, _ in gs], pairs, got, 24, 500, [schedule] * len(gs))
    # the same requests in another order, twice, on the same runtime
    got2 = rt.decode(pairs[::-1])[::-1]
    _check_same(torch, got2, want)
    rt.close()
    for _, G in gs:
        G.close()


def test_ragged_latency_variant(torch_cuda):
    """A ragged round whose items all reside at once (FP32, serial, global
    slabs) runs the variant with the deeper prefetch ring; each request
    equals its single decode on the persistent kernel (forced by a grid
    below the item count) bit for bit, eagerly and in captured replays."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    gs = _graphs()
    sizes = [3, 1, 2, 5]
    pairs = [(G, _dev(torch, sample(dem, B, 190 + i).syndromes)) for i, ((dem, G), B) in enumerate(zip(gs, sizes))]
    want = []
    for (dem, G), (_, s), B in zip(gs, pairs, sizes):
        G.set_launch(slab_in_lds=0, grid=max(1, B * G.info()["L"] // 2))
        want.append(G.decode(s))
        G.set_launch()
    rt = P.Runtime()
    _check_same(torch, rt.decode(pairs), want)
    ex = P.Exec(pairs)
    for _ in range(3):
        outs = ex.launch()
        torch.cuda.synchronize()
        snap = [tuple(t.clone() for t in o) for o in outs]
        rt.decode([(G, s.clone()) for G, s in pairs])  # eager work between replays
        torch.cuda.synchronize()
        _check_same(torch, snap, want)
    ex.close()
    rt.close()
    for _, G in gs:
        G.close()


def test_ragged_mixed_schedules(torch_cuda):
    """Serial, parallel (BP+LSD-0) and layered graphs in one ragged call
    share one persistent launch; every request still equals its single
    decode, in either order; a serial + layered call (no parallel segment)
    as well."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    ser, par = _graphs("serial"), _graphs("parallel")
    lay = []
    for i, dem in enumerate((code_capacity_dem(5, 0.05), circuit_dem(5, 5, 1e-3))):
        lay.append((dem, P.Graph.from_dem(dem, permutations(dem.m, 8, 60 + i), L=8, M=3, T_max=20,
                                          schedule="layered")))
    gs = [ser[0], par[1], lay[0], ser[3], par[2], lay[1], par[0]]
    sizes = [500, 300, 200, 64, 1, 100, 200]
    pairs = [(G, _dev(torch, sample(dem, B, 120 + i).syndromes)) for i, ((dem, G), B) in enumerate(zip(gs, sizes))]
    want = [G.decode(s) for G, s in pairs]
    rt = P.Runtime()
    got = rt.decode(pairs)
    _check_same(torch, got, want)
    kinds = ["serial", "parallel", "layered", "serial", "parallel", "layered", "parallel"]
    _check_oracle([dem for dem, _ in gs], pairs, got, 16, 600, kinds)
    _check_same(torch, rt.decode(pairs[::-1])[::-1], want)
    sl = [pairs[0], pairs[2], pairs[3], pairs[5]]
    _check_same(torch, rt.decode(sl), [want[0], want[2], want[3], want[5]])
    rt.close()
    for _, G in ser + par + lay:
        G.close()


def test_ragged_benchmark_graph_mix(torch_cuda):
    """The d = 9 benchmark graph with smaller codes in one launch."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dems = [circuit_dem(9, 9, 1e-3), circuit_dem(5, 5, 1e-3), code_capacity_dem(5, 0.05)]
    gs = [P.Graph.from_dem(d, permutations(d.n, 32 if i < 2 else 16, 60 + i), L=32 if i < 2 else 16, M=5,
                           T_max=20 if i < 2 else 32) for i, d in enumerate(dems)]
    pairs = [(G, _dev(torch, sample(d, B, 70 + i).syndromes)) for i, (d, G, B) in enumerate(zip(dems, gs, [256, 512, 2000]))]
    want = [G.decode(s) for G, s in pairs]
    rt = P.Runtime()
    got = rt.decode(pairs)
    _check_same(torch, got, want)
    _check_oracle(dems, pairs, got, 12, 700)
    rt.close()
    for G in gs:
        G.close()


def test_exec_replays_match_eager(torch_cuda):
    """A captured sequence, replayed several times with eager work and
    synchronisations between the replays and the syndrome buffers refilled;
    every replay must equal the eager result on the same contents."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    gs = _graphs()
    sizes = [512, 64, 300, 128]
    bufs = [(G, _dev(torch, sample(dem, B, 100 + i).syndromes)) for i, ((dem, G), B) in enumerate(zip(gs, sizes))]
    ex = P.Exec(bufs)
    rt = P.Runtime()
    for rep in range(4):
        if rep >= 2:  # new syndromes in the same buffers
            for i, ((dem, G), (_, s)) in enumerate(zip(gs, bufs)):
                s.copy_(_dev(torch, sample(dem, s.shape[0], 200 + 10 * rep + i).syndromes))
        outs = ex.launch()
        torch.cuda.synchronize()
        snap = [tuple(t.clone() for t in o) for o in outs]
        eager = rt.decode([(G, s.clone()) for G, s in bufs])  # eager work between replays
        torch.cuda.synchronize()
        _check_same(torch, snap, eager)
        single = [G.decode(s) for G, s in bufs]
        _check_same(torch, snap, single)
        if rep in (0, 3):
            _check_oracle([dem for dem, _ in gs], bufs, snap, 12, 800 + rep)
    ex.close()
    rt.close()
    for _, G in gs:
        G.close()


def test_autotune_keeps_results(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    for dem, L, M, T in [(phenomenological_dem(11, 11, 0.01, 0.01), 32, 5, 50), (circuit_dem(7, 7, 1e-3), 32, 5, 20)]:
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 5), L=L, M=M, T_max=T)
        s = _dev(torch, sample(dem, 1500, 6).syndromes)
        c1, o1, s1 = G.decode(s)
        ch = G.autotune(s[:512])
        assert ch["slab_in_lds"] in (0, 1) and ch["grid"] >= 0 and ch["shots_per_wave"] in (1, 2, 4)
        print(f"autotune {dem.name}: {ch}", flush=True)
        c2, o2, s2 = G.decode(s)
        assert torch.equal(c1, c2) and torch.equal(o1, o2) and torch.equal(s1[:, DET], s2[:, DET])
        G.close()
