"""Launch settings of K1 (through the C ABI): several shots per wavefront
and decisions in global memory.

With shots_per_wave = P > 1 one wavefront runs P shots of a member side by
side on the member's schedule recut into chunks of 64 / P edges.  The recut
keeps the sweep (a part of a set of independent columns is independent, and
the order of the 64-edge chunks is kept), and every message is computed by
the same operations in the same order, so the outputs must equal those of
one shot per wavefront bit for bit, in FP32 and FP64 alike, for batches
that do not fill the last group of P shots.  Decisions kept in global
memory (per-chunk masks and a bitmap) instead of LDS change only where the
same bits are stored, so they too must give identical outputs.  The FP64
decodes are also compared with the oracle on a sample of shots (Sec.
III.D.2; Algorithm 1's serial sweep).  The same holds in ragged launches
that mix graphs with different settings, in captured replays and in the
no-allocation entry point.
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


SPECS = [
    ("code capacity d=5", lambda: code_capacity_dem(5, 0.05), 16, 5, 32),
    ("circuit d=5", lambda: circuit_dem(5, 5, 1e-3), 32, 5, 20),
    ("phenomenological d=7", lambda: phenomenological_dem(7, 7, 0.01, 0.01), 24, 5, 30),
    ("circuit d=7", lambda: circuit_dem(7, 7, 1e-3), 32, 5, 20),
]


def _same(torch, a, b):
    (c1, o1, s1), (c2, o2, s2) = a, b
    assert torch.equal(c1, c2)
    assert torch.equal(o1, o2)
    assert torch.equal(s1[:, DET], s2[:, DET])


@pytest.mark.parametrize("bits", [32, 64])
def test_multishot_equals_one_shot_per_wave(torch_cuda, bits):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    for i, (label, mk, L, M, T) in enumerate(SPECS):
        dem = mk()
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 60 + i), L=L, M=M, T_max=T, message_bits=bits)
        synd = sample(dem, 301, 70 + i).syndromes  # 301 = 4 * 75 + 1: the last group is ragged
        s = _dev(torch, synd)
        G.set_launch(slab_in_lds=0, shots_per_wave=1, decisions_global=0)
        ref = G.decode(s)
        # the slab in LDS (where it fits: the code-capacity and d = 7
        # phenomenological graphs), then the global-slab settings
        for lds, Pw, dec in ((1, 1, 0), (0, 1, 1), (0, 2, 0), (0, 2, 1), (0, 4, 0), (0, 4, 1)):
            G.set_launch(slab_in_lds=lds, shots_per_wave=Pw, decisions_global=dec)
            got_l = G.get_launch()
            assert (got_l["shots_per_wave"], got_l["decisions_global"]) == (Pw, dec)
            got = G.decode(s)
            _same(torch, got, ref)
            # batches smaller than one group
            for B in (1, 2, 3):
                _same(torch, G.decode(s[:B].contiguous()), tuple(x[:B] for x in ref))
        torch.cuda.synchronize()
        e = P.unpack_bits(got[0], dem.n)
        st = got[2].cpu().numpy()
        check_valid(dem, e, synd, st)
        if bits == 64:
            print(sampled_oracle_parity(dem, G, synd, e, st, 40, 90 + i, f"{label} P=4"), flush=True)
        G.close()


def test_latency_variant_equals_persistent(torch_cuda):
    """A launch whose work items all reside at once runs the variant of K1
    with the deeper prefetch ring (FP32, serial schedule, global slab, one
    shot per wavefront, decisions in LDS); it loads the same chunks ahead of
    the same operations, so its outputs equal those of the persistent kernel
    bit for bit.  A grid below the item count forces the persistent one."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    for i, (label, mk, L, M, T) in enumerate(SPECS):
        dem = mk()
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 160 + i), L=L, M=M, T_max=T)
        s = _dev(torch, sample(dem, 64, 170 + i).syndromes)
        for B in (1, 3, 64):
            sb = s[:B].contiguous()
            G.set_launch(slab_in_lds=0, shots_per_wave=1, decisions_global=0)
            fast = G.decode(sb)
            G.set_launch(slab_in_lds=0, grid=max(1, B * L // 2), shots_per_wave=1, decisions_global=0)
            _same(torch, fast, G.decode(sb))
        G.close()


def test_multishot_schedule_shape(torch_cuda):
    """The recut schedule of a graph whose 64-edge chunks are far from full
    needs fewer chunk steps per shot: for the d = 5 circuit graph, 4 shots
    per wavefront on 16-edge chunks take well under the 64-edge chunk count
    per shot (this is what the autotuner trades against the slower steps)."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(5, 5, 1e-3)
    G = P.Graph.from_dem(dem, permutations(dem.n, 8, 3), L=8, M=5, T_max=20)
    info = G.info()
    assert info["nnz"] < 0.5 * 64 * info["chunks_max"]  # chunks far from full
    G.set_launch(shots_per_wave=4)
    s = _dev(torch, sample(dem, 64, 4).syndromes)
    c, o, st = G.decode(s)
    torch.cuda.synchronize()
    check_valid(dem, P.unpack_bits(c, dem.n), s.cpu().numpy(), st.cpu().numpy())
    G.close()


def test_multishot_in_ragged_capture_and_noalloc(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    gs, ss = [], []
    for i, (label, mk, L, M, T) in enumerate(SPECS):
        dem = mk()
        G = P.Graph.from_dem(dem, permutations(dem.n, L, 60 + i), L=L, M=M, T_max=T)
        gs.append((dem, G))
        ss.append(_dev(torch, sample(dem, [37, 150, 5, 64][i], 80 + i).syndromes))
    # one graph per setting, plus a layered one in the same launch
    for (_, G), Pw, dec in zip(gs, (4, 2, 1, 4), (0, 1, 1, 0)):
        G.set_launch(shots_per_wave=Pw, decisions_global=dec)
    demL = circuit_dem(5, 5, 1e-3)
    GL = P.Graph.from_dem(demL, permutations(demL.m, 16, 9), L=16, M=5, T_max=20, schedule="layered")
    sL = _dev(torch, sample(demL, 40, 10).syndromes)
    pairs = [(G, s) for (_, G), s in zip(gs, ss)] + [(GL, sL)]
    single = [G.decode(s) for G, s in pairs]
    rt = P.Runtime()
    got = rt.decode(pairs)
    for a, b in zip(got, single):
        _same(torch, a, b)
    ex = P.Exec(pairs)
    for rep in range(3):
        ex.launch()
        torch.cuda.synchronize()
        for a, b in zip(ex.outs, single):
            _same(torch, a, b)
    ex.close()
    rt.close()
    # the no-allocation entry point runs the chosen setting too
    for (_, G), s, want in zip(gs, ss, single):
        _same(torch, G.decode(s, noalloc=True), want)
    # every serial graph on one shot per wavefront: a launch of the plain
    # ragged kernel with decisions in global memory for all of them
    for (_, G), dec in zip(gs, (1, 0, 0, 0)):
        G.set_launch(shots_per_wave=1, decisions_global=dec)
    pairs2 = [(G, s) for (_, G), s in zip(gs, ss)]
    for a, b in zip(P.Runtime().decode(pairs2), single[:4]):
        _same(torch, a, b)
    for _, G in gs:
        G.close()
    GL.close()


def test_autotune_choices_and_shape_cache(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(5, 5, 1e-3)
    perms = permutations(dem.n, 32, 21)
    G1 = P.Graph.from_dem(dem, perms, L=32, M=5, T_max=20)
    s = _dev(torch, sample(dem, 2048, 22).syndromes)
    ref = G1.decode(s)
    ch = G1.autotune(s)
    assert ch["shots_per_wave"] in (1, 2, 4) and ch["grid"] >= 0 and ch["slab_in_lds"] in (0, 1)
    assert not ch["from_cache"] and ch["ms"] > 0
    assert G1.get_launch()["shots_per_wave"] == ch["shots_per_wave"]
    _same(torch, G1.decode(s), ref)
    # a second graph of the same shape takes the cached choice untimed
    G2 = P.Graph.from_dem(dem, perms, L=32, M=5, T_max=20)
    ch2 = G2.autotune(s)
    assert ch2["from_cache"]
    assert (ch2["shots_per_wave"], ch2["grid"], ch2["slab_in_lds"]) == \
        (ch["shots_per_wave"], ch["grid"], ch["slab_in_lds"])
    _same(torch, G2.decode(s), ref)
    print(f"autotune d=5 circuit, 2048 shots: {ch}", flush=True)
    G1.close()
    G2.close()


def test_set_launch_rejects_what_it_cannot_run(torch_cuda):
    import paper_2508_15743_amd as P

    dem = code_capacity_dem(5, 0.05)
    G = P.Graph.from_dem(dem, permutations(dem.n, 4, 1), L=4, M=2, T_max=10)
    with pytest.raises(P.VibeError) as e:
        G.set_launch(shots_per_wave=3)
    assert e.value.code == P.VIBE_EINVAL
    with pytest.raises(P.VibeError) as e:
        G.set_launch(slab_in_lds=1, shots_per_wave=2)
    assert e.value.code == P.VIBE_EINVAL
    with pytest.raises(P.VibeError) as e:
        G.set_launch(slab_in_lds=1, decisions_global=1)
    assert e.value.code == P.VIBE_EINVAL
    Gp = P.Graph.from_dem(dem, permutations(dem.n, 1, 1), L=1, M=1, T_max=10, schedule="parallel")
    with pytest.raises(P.VibeError) as e:
        Gp.set_launch(shots_per_wave=2)
    assert e.value.code == P.VIBE_EUNSUPPORTED
    # a failed call leaves the setting as it was
    assert G.get_launch()["shots_per_wave"] == 1
    G.close()
    Gp.close()


def test_decisions_global_parallel_schedule_and_ragged(torch_cuda):
    """Decisions in global memory on the parallel (flooding) schedule, alone
    and in a ragged launch mixing it with a serial graph: identical to the
    decisions in LDS."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dems = [circuit_dem(5, 5, 1e-3), phenomenological_dem(7, 7, 0.01, 0.01)]
    Gp = P.Graph.from_dem(dems[0], permutations(dems[0].n, 1, 31), L=1, M=1, T_max=20, schedule="parallel")
    Gs = P.Graph.from_dem(dems[1], permutations(dems[1].n, 24, 32), L=24, M=5, T_max=30)
    ss = [_dev(torch, sample(d, 333, 40 + i).syndromes) for i, d in enumerate(dems)]
    for G in (Gp, Gs):
        G.set_launch(decisions_global=0)
    ref = [Gp.decode(ss[0]), Gs.decode(ss[1])]
    for G in (Gp, Gs):
        G.set_launch(decisions_global=1)
    _same(torch, Gp.decode(ss[0]), ref[0])
    _same(torch, Gs.decode(ss[1]), ref[1])
    rt = P.Runtime()
    for a, b in zip(rt.decode([(Gp, ss[0]), (Gs, ss[1])]), ref):
        _same(torch, a, b)
    rt.close()
    Gp.close()
    Gs.close()


@pytest.mark.parametrize("bits", [32, 64])
def test_settings_on_unusual_inputs(torch_cuda, bits):
    """Priors above 1/2 (the zero-syndrome shortcut off), columns in no
    check, zero syndromes, a per-iteration scaling table, and the
    correction limits M = 1 and M = L: every launch setting gives the
    outputs of the default one, and the FP64 decode is the oracle's."""
    import paper_2508_15743_amd as P
    from oracle import oracle as O
    from synth.dem import dem_from_dense

    torch = torch_cuda
    base = code_capacity_dem(5, 0.05)
    H = np.concatenate([base.dense_h(), np.zeros((base.m, 2), np.uint8)], axis=1)
    rng = np.random.default_rng(151)
    pri = rng.uniform(0.02, 0.3, H.shape[1])
    pri[[2, 7, 19]] = [0.6, 0.75, 0.55]
    lobs = np.concatenate([base.dense_l(), np.zeros((base.dense_l().shape[0], 2), np.uint8)], axis=1)
    dem = dem_from_dense(H, pri, lobs)
    synd = sample(dem, 203, 152).syndromes
    synd[:7] = 0  # zero syndromes at the head of the batch
    s = _dev(torch, synd)
    for M in (1, 5, 16):
        perms = permutations(dem.n, 16, 153 + M)
        G = P.Graph.from_dem(dem, perms, L=16, M=M, T_max=24, message_bits=bits)
        G.set_alpha(np.linspace(0.5, 0.9, 24))
        G.set_launch(slab_in_lds=1)
        ref = G.decode(s)
        for lds, Pw, dec in ((0, 1, 0), (0, 1, 1), (0, 2, 1), (0, 4, 0)):
            G.set_launch(slab_in_lds=lds, shots_per_wave=Pw, decisions_global=dec)
            _same(torch, G.decode(s), ref)
        if bits == 64:
            want = O.decode(O.OracleGraph(dem), G.schedules(), synd, L=16, M=M, T=24,
                            alpha=np.linspace(0.5, 0.9, 24), threads=8)
            e = P.unpack_bits(ref[0], dem.n)
            assert (want["ehat"] == e).all(1).mean() >= 0.999
        G.close()
