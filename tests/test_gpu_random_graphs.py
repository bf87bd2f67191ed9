"""Randomly structured graphs against the oracle, FP64 bit for bit (Alg. 1
serial and parallel branches for the members; Sec. III.D.2 for whole
decodes), and the FP32 decode to the FP32 bar.

The workloads' graphs are regular: column degrees of a few checks, row
degrees up to ~130, priors in a narrow band.  These graphs draw the
structure at random instead, seeded: column degrees from 0 (a column in no
check) up to the supported 15, one or two dense rows that touch most
columns (a row spanning many 64-edge chunks), isolated checks, priors from
1e-5 up to 0.6 (above one half the channel LLR is negative), one to three
observables, and ensembles from one member to 16 with M from 1 to L and
T from 1 to 20, on the serial, parallel and layered schedules.  The
launch settings (several shots per wavefront, decisions in global memory)
and a ragged launch over several of them must leave every output
unchanged.
"""
import numpy as np
import pytest

from synth.dem import dem_from_columns
from synth.sample import permutations, sample

from parity_helpers import NT, check_valid, fp32_decode_bar

pytestmark = pytest.mark.gpu


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


def random_dem(seed):
    """A seeded random detector error model (see the module docstring)."""
    rng = np.random.default_rng(seed)
    m = int(rng.integers(8, 400))
    n = int(rng.integers(m // 2 + 8, 4 * m))
    degs = rng.choice([0, 1, 2, 3, 4, 6, 15], size=n, p=[0.02, 0.2, 0.35, 0.2, 0.12, 0.08, 0.03])
    cols = [set(rng.choice(m, size=min(int(d), m), replace=False).tolist()) for d in degs]
    for r in rng.choice(m, size=int(rng.integers(1, 3)), replace=False):
        for v in np.flatnonzero(rng.random(n) < 0.6):
            if 0 < len(cols[v]) < 15:
                cols[v].add(int(r))
    k = int(rng.integers(1, 4))
    obs = [[o for o in range(k) if rng.random() < 0.1] for _ in range(n)]
    priors = 10.0 ** rng.uniform(-5, -0.7, n)
    hi = rng.random(n) < 0.02
    priors[hi] = rng.uniform(0.5, 0.6, int(hi.sum()))
    return dem_from_columns(m, k, [sorted(c) for c in cols], obs, priors, name=f"random graph {seed}")


SHAPES = [(1, 1, 20), (3, 2, 7), (8, 8, 1), (16, 5, 20), (16, 1, 2), (8, 3, 20)]


@pytest.mark.parametrize("seed", range(12))
def test_random_graph_fp64_bit_exact(torch_cuda, seed):
    import paper_2508_15743_amd as P
    from oracle import oracle as O

    torch = torch_cuda
    dem = random_dem(1000 + seed)
    L, M, T = SHAPES[seed % len(SHAPES)]
    perms = permutations(dem.n, L, 2000 + seed)
    G = P.Graph.from_dem(dem, perms, L=L, M=M, T_max=T, message_bits=64)
    synd = sample(dem, 96, 3000 + seed).syndromes
    s = _dev(torch, synd)
    g = O.OracleGraph(dem)
    print(f"{dem.name}: m={dem.m} n={dem.n} nnz={dem.nnz} k={dem.k} "
          f"max row degree {dem.summary()['max_row_degree']}, L={L} M={M} T={T}", flush=True)
    # members (stop on convergence), on the first shots
    tc, post, eh = G.bp_ensemble(s[:6].contiguous(), T_run=T, stop=True)
    tc, post, eh = tc.cpu().numpy(), post.cpu().numpy(), P.unpack_bits(eh, dem.n)
    for i in range(6):
        for j in range(L):
            r = O.bp(g, synd[i], perm=perms[j], T=T, stop=True)
            assert r["t_conv"] == tc[i, j], (i, j)
            assert np.array_equal(r["ehat"], eh[i, j]), (i, j)
            assert np.array_equal(r["post"], post[i, j]), (i, j)
    # whole decodes, every shot
    ref = O.decode(g, G.schedules(), synd, L=L, M=M, T=T, threads=NT)
    c, o, st = G.decode(s)
    torch.cuda.synchronize()
    e, o, st = P.unpack_bits(c, dem.n), o.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(e, ref["ehat"]), np.flatnonzero((e != ref["ehat"]).any(1))[:10]
    assert np.array_equal(o[:, :dem.k], ref["obs"])
    assert np.array_equal(st[:, 0] & 7, ref["rec"][:, 0].astype(np.int64) & 7)
    check_valid(dem, e, synd, st)
    # launch settings leave every output unchanged
    want = (c, torch.from_numpy(o).to("cuda:0"))
    for Pw, dec in ((2, 0), (4, 1), (1, 1)):
        G.set_launch(shots_per_wave=Pw, decisions_global=dec)
        c2, o2, _ = G.decode(s)
        assert torch.equal(c2, want[0]) and torch.equal(o2, want[1]), (Pw, dec)
    G.close()
    # the parallel schedule: one member
    Gp = P.Graph.from_dem(dem, permutations(dem.n, 1, 1), L=1, M=1, T_max=T, message_bits=64,
                          schedule="parallel")
    refp = O.decode(g, Gp.schedules(), synd, L=1, M=1, T=T, threads=NT, schedule="parallel")
    cp, op, stp = Gp.decode(s)
    assert np.array_equal(P.unpack_bits(cp, dem.n), refp["ehat"])
    Gp.close()
    # the layered schedule: members sweep the checks in their own orders
    cperm = permutations(dem.m, L, 4000 + seed)
    Gl = P.Graph.from_dem(dem, cperm, L=L, M=M, T_max=T, message_bits=64, schedule="layered")
    refl = O.decode(g, Gl.schedules(), synd, L=L, M=M, T=T, threads=NT, schedule="layered")
    cl, ol, stl = Gl.decode(s)
    assert np.array_equal(P.unpack_bits(cl, dem.n), refl["ehat"])
    Gl.close()


def test_random_graphs_in_one_ragged_round(torch_cuda):
    """Six random graphs of different shapes in one ragged call (one
    persistent launch): every request equals its single decode."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    pairs = []
    for i in range(6):
        dem = random_dem(1200 + i)
        L, M, T = SHAPES[i]
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 2200 + i), L=L, M=M, T_max=T)
        pairs.append((G, _dev(torch, sample(dem, 50 + 37 * i, 3200 + i).syndromes)))
    want = [G.decode(s) for G, s in pairs]
    rt = P.Runtime()
    got = rt.decode(pairs)
    for (c1, o1, _), (c2, o2, _) in zip(got, want):
        assert torch.equal(c1, c2) and torch.equal(o1, o2)
    rt.close()
    for G, _ in pairs:
        G.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_graph_fp32_decode(torch_cuda, seed):
    import paper_2508_15743_amd as P
    from oracle import oracle as O

    torch = torch_cuda
    dem = random_dem(1100 + seed)
    L, M, T = (16, 5, 20)
    perms = permutations(dem.n, L, 2100 + seed)
    G = P.Graph.from_dem(dem, perms, L=L, M=M, T_max=T)
    synd = sample(dem, 400, 3100 + seed).syndromes
    c, o, st = G.decode(_dev(torch, synd))
    torch.cuda.synchronize()
    e, st = P.unpack_bits(c, dem.n), st.cpu().numpy()
    check_valid(dem, e, synd, st)
    ref = O.decode(O.OracleGraph(dem), G.schedules(), synd, L=L, M=M, T=T, threads=NT)
    agree = (ref["ehat"] == e).all(1)
    print(f"{dem.name} FP32: " + fp32_decode_bar(agree, ref["lsd_used"], (st[:, 0] & 2) != 0, ref["min_q_gap"],
                                                 L, dem.n, ref["min_abs_post"]), flush=True)
    G.close()
