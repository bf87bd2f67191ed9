"""The differentiable decoder (vibe_bp_grad) against the oracle.

The loss is the oracle's or_bp_loss summed over shots and ensemble members;
the gradient is checked against the oracle's central differences on every
entry the oracle flags smooth (no argmin, sign or clamp switches within the
step).  In FP64 the unrolled iterations follow the oracle's operation order,
so the loss agrees to rounding and the gradient to the difference quotient's
own error.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth.dem import circuit_dem, code_capacity_dem
from synth.sample import permutations, sample

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15743_amd as P

    P.lib()
    return torch


def _inputs(dem, B, K, seed):
    rng = np.random.default_rng(seed)
    lam = np.log(1 / rng.uniform(0.01, 0.2, dem.n) - 1)  # distinct LLRs: no ties at the first iteration
    alpha = rng.uniform(0.5, 1.0, K)
    synd = sample(dem, B, seed + 1).syndromes
    return lam, alpha, synd


def _oracle(dem, synd, lam, alpha, K, perms, idx=None):
    """Summed loss and FD gradient over shots x members, with the flags
    AND-ed over every item."""
    g = O.OracleGraph(dem)
    loss, dl, da = 0.0, np.zeros(dem.n), np.zeros(K)
    okl, oka = np.ones(dem.n, bool), np.ones(K, bool)
    for s in synd:
        for perm in (perms if perms is not None else [None]):
            loss += O.bp_loss(g, s, lam, alpha, K, perm)[0]
            a, b, c, d = O.fd_grad(g, s, lam, alpha, K, perm, idx=idx)
            dl += a
            da += c
            okl &= b
            oka &= d
    if idx is not None:
        sel = np.zeros(dem.n, bool)
        sel[idx] = True
        okl &= sel
    return loss, dl, okl, da, oka


def _graph(P, dem, L, schedule, bits, seed=3):
    perms = permutations(dem.n, L, seed)
    G = P.Graph.from_dem(dem, perms, L=L, M=1, T_max=8, schedule=schedule, message_bits=bits)
    return G, (perms if schedule == "serial" else None)


def _run(torch, G, synd, lam, alpha, bits=64):
    dt = torch.float64 if bits == 64 else torch.float32
    loss, dl, da = G.bp_grad(torch.from_numpy(synd).cuda(), torch.tensor(lam, dtype=dt),
                             torch.tensor(alpha, dtype=dt))
    return loss.item(), dl.cpu().numpy(), da.cpu().numpy()


def _close(got, want, ok, tol):
    assert ok.sum() > 0
    err = np.abs(got - want)[ok] / np.maximum(1.0, np.abs(want)[ok])
    assert err.max() <= tol, (err.max(), int(np.argmax(err)))


@pytest.mark.parametrize("schedule,L", [("serial", 4), ("parallel", 1)])
def test_grad_fp64_code_capacity(torch_cuda, schedule, L):
    import paper_2508_15743_amd as P

    dem = code_capacity_dem(5, 0.08)
    K = 6
    lam, alpha, synd = _inputs(dem, 5, K, 11)
    G, perms = _graph(P, dem, L, schedule, 64)
    loss, dl, da = _run(torch_cuda, G, synd, lam, alpha)
    wl, wdl, okl, wda, oka = _oracle(dem, synd, lam, alpha, K, perms)
    assert abs(loss - wl) <= 1e-12 * max(1.0, abs(wl))
    assert okl.mean() >= 0.8 and oka.all()
    _close(dl, wdl, okl, 1e-6)
    _close(da, wda, oka, 1e-6)
    G.close()


@pytest.mark.parametrize("schedule,L", [("serial", 2), ("parallel", 1)])
def test_grad_fp64_circuit(torch_cuda, schedule, L):
    """The d = 5 circuit-level graph (several chunks per member, columns of
    degree up to the graph's maximum): all alpha entries and a sample of 48
    columns."""
    import paper_2508_15743_amd as P

    dem = circuit_dem(5, 5, 2e-3)
    K = 5
    lam, alpha, synd = _inputs(dem, 2, K, 21)
    idx = np.random.default_rng(5).choice(dem.n, 48, replace=False)
    G, perms = _graph(P, dem, L, schedule, 64)
    loss, dl, da = _run(torch_cuda, G, synd, lam, alpha)
    wl, wdl, okl, wda, oka = _oracle(dem, synd, lam, alpha, K, perms, idx)
    assert abs(loss - wl) <= 1e-12 * max(1.0, abs(wl))
    assert okl.sum() >= 36 and oka.sum() >= K - 2
    _close(dl, wdl, okl, 1e-6)
    _close(da, wda, oka, 1e-6)
    G.close()


def test_grad_fp32_against_oracle(torch_cuda):
    """FP32 messages: loss to single-precision rounding, gradient to a bound
    of the accumulated rounding over K iterations."""
    import paper_2508_15743_amd as P

    dem = code_capacity_dem(7, 0.08)
    K = 6
    lam, alpha, synd = _inputs(dem, 6, K, 31)
    G, perms = _graph(P, dem, 4, "serial", 32)
    loss, dl, da = _run(torch_cuda, G, synd, lam, alpha, bits=32)
    wl, wdl, okl, wda, oka = _oracle(dem, synd, lam, alpha, K, perms)
    assert abs(loss - wl) <= 1e-4 * max(1.0, abs(wl))
    _close(dl, wdl, okl, 2e-3)
    _close(da, wda, oka, 2e-3)
    G.close()


def test_grad_deterministic_and_autograd(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(5, 5, 2e-3)
    K = 4
    lam, alpha, synd = _inputs(dem, 64, K, 41)
    G, _ = _graph(P, dem, 8, "serial", 32)
    s = torch.from_numpy(synd).cuda()
    r1 = G.bp_grad(s, torch.tensor(lam), torch.tensor(alpha))
    r2 = G.bp_grad(s, torch.tensor(lam), torch.tensor(alpha))
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)
    lam_t = torch.tensor(lam, dtype=torch.float32, device="cuda:0", requires_grad=True)
    al_t = torch.tensor(alpha, dtype=torch.float32, device="cuda:0", requires_grad=True)
    loss = P.bp_loss(G, s, lam_t, al_t)
    (2.0 * loss).backward()
    assert torch.allclose(loss.double(), r1[0][0], rtol=1e-6)
    assert torch.equal(lam_t.grad, (2.0 * r1[1].float()))
    assert torch.equal(al_t.grad, (2.0 * r1[2].float()))
    G.close()


def test_grad_rejects_bad_arguments(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = code_capacity_dem(5, 0.05)
    G, _ = _graph(P, dem, 2, "serial", 32)
    s = torch.zeros((3, dem.m), dtype=torch.uint8, device="cuda:0")
    lam = torch.ones(dem.n)
    with pytest.raises(P.VibeError):
        G.bp_grad(s, lam, torch.ones(0))  # K = 0
    with pytest.raises(P.VibeError):
        G.bp_grad(s, lam, torch.ones(65))  # K > 64
    with pytest.raises(P.VibeError):
        G.bp_grad(s, lam, torch.ones(3), eps=0.0)
    with pytest.raises(ValueError):
        G.bp_grad(s, torch.ones(dem.n + 1), torch.ones(3))
    G.close()


def test_grad_full_size_additive_and_sampled(torch_cuda):
    """The configuration the benchmark times: d = 5 circuit-level graph,
    L = 32 serial members, K = 16, FP32, 4096 shots, alpha_t = 0.625 and
    lambda from the priors.  Every per-item result is independent of the
    launch, so the batch equals the sum of its four quarters up to the order
    of the FP64 sums; two sampled shots alone match the oracle's loss."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(5, 5, 1e-3)
    K, L, B = 16, 32, 4096
    perms = permutations(dem.n, L, 7)
    G = P.Graph.from_dem(dem, perms, L=L, M=5, T_max=20)
    synd = sample(dem, B, 8).syndromes
    s = torch.from_numpy(synd).cuda()
    lam = np.log((1 - dem.priors) / dem.priors)
    lam_t = torch.tensor(lam, dtype=torch.float32)
    al_t = torch.full((K,), 0.625)
    loss, dl, da = G.bp_grad(s, lam_t, al_t)
    assert torch.isfinite(dl).all() and torch.isfinite(da).all()
    parts = [G.bp_grad(s[q * 1024:(q + 1) * 1024], lam_t, al_t) for q in range(4)]
    for i, full in enumerate((loss, dl, da)):
        summed = sum(p[i] for p in parts)
        scale = float(torch.abs(torch.stack([p[i] for p in parts])).sum(0).max())
        assert float(torch.abs(full - summed).max()) <= 1e-12 * max(scale, 1.0)
    rows = np.random.default_rng(9).choice(B, 2, replace=False)
    got = G.bp_grad(s[rows], lam_t, al_t)[0].item()
    g = O.OracleGraph(dem)
    want = sum(O.bp_loss(g, synd[r], lam, np.full(K, 0.625), K, perm)[0] for r in rows for perm in perms)
    assert abs(got - want) <= 1e-4 * max(1.0, abs(want))
    G.close()


@pytest.mark.parametrize("bits,schedule", [(64, "serial"), (32, "serial"), (64, "parallel"), (32, "parallel")])
def test_grad_same_at_every_chunk_width(torch_cuda, bits, schedule):
    """The gradient schedule may run 1, 2 or 4 shots per wavefront (chunk
    widths 64, 32, 16).  Per-item arithmetic is the same at every width, so
    the sums agree up to their order; the d = 5 circuit graph with an odd
    number of shots also leaves idle items in the last wavefront."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(5, 5, 2e-3)
    K = 6
    lam, alpha, synd = _inputs(dem, 37, K, 51)
    G, _ = _graph(P, dem, 8 if schedule == "serial" else 1, schedule, bits)
    dt = torch.float64 if bits == 64 else torch.float32
    s = torch.from_numpy(synd).cuda()
    res = {}
    for w in (64, 32, 16):
        G.set_grad_width(w)
        res[w] = [x.cpu().numpy() for x in G.bp_grad(s, torch.tensor(lam, dtype=dt), torch.tensor(alpha, dtype=dt))]
        assert G.info()["grad_width"] == w
    for w in (32, 16):
        for got, want in zip(res[w], res[64]):
            scale = max(1.0, float(np.abs(want).max()))
            assert np.abs(got - want).max() <= 1e-9 * scale
    G.set_grad_width(0)
    with pytest.raises(P.VibeError):
        G.set_grad_width(24)
    G.close()


def test_fit_lowers_the_loss_and_gives_a_valid_decoder(torch_cuda):
    """The fitting loop over the channel LLRs and one shared scaling factor
    (Adam on the gradient kernel's output): on the d = 5 circuit graph with
    8 unrolled iterations the loss falls below the starting one, the
    returned parameters are those of the lowest loss seen, the scaling
    factor stays in its range, and a decoder built from the fitted priors
    returns corrections that satisfy H e = s on every shot LSD did not
    flag."""
    import paper_2508_15743_amd as P
    from paper_2508_15743_amd import tune

    torch = torch_cuda
    dem = circuit_dem(5, 5, 1e-3)
    perms = permutations(dem.n, 4, 71)
    G = P.Graph.from_dem(dem, perms, L=4, M=1, T_max=8)
    s = torch.from_numpy(sample(dem, 512, 72).syndromes).cuda()
    lam0 = np.log((1 - dem.priors) / dem.priors)
    lam, alpha, losses = tune.fit(G, s, 8, steps=12, lam0=lam0)
    assert len(losses) == 13 and min(losses) < 0.97 * losses[0], losses
    got = float(G.bp_grad(s, torch.tensor(lam), torch.full((8,), alpha))[0].item()) / 512
    assert abs(got - min(losses)) <= 1e-4 * min(losses), (got, min(losses))
    assert 0.05 <= alpha <= 1.0 and np.all(np.isfinite(lam)) and lam.min() >= 1e-3
    G.close()
    pri = tune.priors_from_llr(lam)
    np.testing.assert_allclose(np.log((1 - pri) / pri), lam, rtol=1e-9)
    Gf = P.Graph(dem.h_indptr, dem.h_indices, pri, dem.l_indptr, dem.l_indices, perms, m=dem.m, n=dem.n,
                 L=4, M=2, T_max=20, alpha=alpha)
    b = sample(dem, 256, 73)
    corr, obs, st = Gf.decode(torch.from_numpy(b.syndromes).cuda())
    e, st = P.unpack_bits(corr, dem.n), st.cpu().numpy()
    ok = (st[:, 0] & 4) == 0
    H = dem.dense_h().astype(np.int64)
    assert np.array_equal((e[ok].astype(np.int64) @ H.T) % 2, b.syndromes[ok])
    Gf.close()


def test_grad_on_the_d17_graph(torch_cuda):
    """The d = 17 circuit-level graph (m = 3672): the gradient kernel's row
    state (88 KB of LDS at one shot per wavefront) needs the large-LDS launch
    and rules out several shots per wavefront.  Two shots and two members,
    K = 4: the FP32 loss matches the oracle's, and the gradient is finite."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = circuit_dem(17, 17, 1e-3)
    K, L = 4, 2
    perms = permutations(dem.n, L, 91)
    G = P.Graph.from_dem(dem, perms, L=L, M=1, T_max=K)
    synd = sample(dem, 2, 92).syndromes
    lam = np.log((1 - dem.priors) / dem.priors)
    alpha = np.full(K, 0.625)
    loss, dl, da = G.bp_grad(torch.from_numpy(synd).cuda(), torch.tensor(lam, dtype=torch.float32),
                             torch.tensor(alpha, dtype=torch.float32))
    assert G.info()["grad_width"] == 64
    assert torch.isfinite(dl).all() and torch.isfinite(da).all()
    g = O.OracleGraph(dem)
    want = sum(O.bp_loss(g, s, lam, alpha, K, perm)[0] for s in synd for perm in perms)
    assert abs(loss.item() - want) <= 1e-4 * max(1.0, abs(want)), (loss.item(), want)
    G.close()


_K16 = {}


def _k16_reference():
    """The oracle's loss and FD gradient for the K = 16 benchmark
    configuration, computed once (the items run on a thread pool; the
    oracle releases the interpreter while it computes)."""
    from concurrent.futures import ThreadPoolExecutor

    if _K16:
        return _K16
    dem = circuit_dem(5, 5, 1e-3)
    K, L = 16, 32
    perms = permutations(dem.n, L, 2030)  # the benchmark's gradient schedules
    synd = sample(dem, 4096, 2031).syndromes[:2]
    # lambda from the priors, moved by up to 1e-3 relative: uniform priors
    # tie many messages exactly, and every alpha_t then switches an argmin
    # between a new and an old message somewhere, so no alpha_t would be
    # smooth; the small move puts the point inside a smooth piece
    rng = np.random.default_rng(2032)
    lam = np.log((1 - dem.priors) / dem.priors) * (1.0 + 1e-3 * rng.uniform(-1.0, 1.0, dem.n))
    alpha = np.full(K, 0.625)
    idx = np.sort(np.random.default_rng(17).choice(dem.n, 64, replace=False))
    g = O.OracleGraph(dem)
    items = [(s, perm) for s in synd for perm in perms]

    def one(it):
        s, perm = it
        f = O.bp_loss(g, s, lam, alpha, K, perm)[0]
        return (f,) + O.fd_grad(g, s, lam, alpha, K, perm, idx=idx)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, items))
    sel = np.zeros(dem.n, bool)
    sel[idx] = True
    _K16.update(dem=dem, K=K, L=L, perms=perms, synd=synd, lam=lam, alpha=alpha,
                loss=sum(r[0] for r in res), dl=sum(r[1] for r in res), da=sum(r[3] for r in res),
                okl=np.logical_and.reduce([r[2] for r in res]) & sel,
                oka=np.logical_and.reduce([r[4] for r in res]))
    return _K16


@pytest.mark.parametrize("bits", [32, 64])
def test_grad_benchmark_configuration_against_finite_differences(torch_cuda, bits):
    """The backward configuration of the workload list at its own depth: the
    d = 5 circuit-level graph, L = 32 serial members, K = 16 unrolled
    iterations, alpha_t = 0.625 and lambda from the priors (moved by up to
    1e-3 relative to break exact ties), on two shots of the benchmark's
    batch (its 131072 items would take the oracle hours).
    The gradient of the summed loss against the oracle's FP64 central
    differences on every alpha_t and on 64 sampled columns, wherever the
    oracle flags the loss smooth in every item: FP64 to 1e-6, FP32 to 2e-3
    (relative to max(1, |value|)).  At least a quarter of the sampled
    columns and half of the alpha_t must be smooth."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    R = _k16_reference()
    dem, K, L = R["dem"], R["K"], R["L"]
    G = P.Graph.from_dem(dem, R["perms"], L=L, M=5, T_max=20, message_bits=bits)
    loss, dl, da = _run(torch, G, R["synd"], R["lam"], R["alpha"], bits=bits)
    G.close()
    okl, oka = R["okl"], R["oka"]
    tol = 1e-6 if bits == 64 else 2e-3
    assert abs(loss - R["loss"]) <= (1e-12 if bits == 64 else 1e-4) * max(1.0, abs(R["loss"])), (loss, R["loss"])
    assert okl.sum() >= 16 and oka.sum() >= K // 2, (okl.sum(), oka.sum())
    _close(dl, R["dl"], okl, tol)
    _close(da, R["da"], oka, tol)
    rel = lambda a, b, ok: float((np.abs(a - b)[ok] / np.maximum(1.0, np.abs(b)[ok])).max())
    print(f"K=16 FP{bits}: loss {loss:.6g} (oracle {R['loss']:.6g}); {int(okl.sum())} of 64 columns and "
          f"{int(oka.sum())} of {K} alpha_t smooth; largest relative error {rel(dl, R['dl'], okl):.2e} "
          f"(lambda), {rel(da, R['da'], oka):.2e} (alpha)", flush=True)
