"""Serving with continuous batching (through the C ABI).

Requests on several resident graphs are submitted from another thread at
irregular times while earlier batches are on the GPU.  Each request's outputs
must equal the single-request decode of the same syndromes bit for bit, and
the server must have formed batches of several requests.  The served
outputs of a sample of shots on every graph are also compared with the FP64
oracle to the FP32 bar of test_gpu_parity.py.
"""
import random
import threading
import time

import numpy as np
import pytest

from synth.dem import circuit_dem, code_capacity_dem, phenomenological_dem
from synth.sample import permutations, sample

from parity_helpers import check_valid, sampled_oracle_parity

pytestmark = pytest.mark.gpu

DET = [0, 1, 2, 4, 5, 6]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15743_amd as P

    P.lib()
    return torch


def test_results_same_alone_and_in_the_mix(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    specs = [(circuit_dem(5, 5, 1e-3), 32, 5, 20), (phenomenological_dem(7, 7, 0.01, 0.01), 24, 5, 30),
             (circuit_dem(7, 7, 1e-3), 32, 5, 20), (code_capacity_dem(5, 0.05), 16, 5, 32)]
    graphs = [P.Graph.from_dem(d, permutations(d.n, L, 80 + i), L=L, M=M, T_max=T)
              for i, (d, L, M, T) in enumerate(specs)]
    rng = random.Random(3)
    reqs = []
    for i in range(150):
        gi = rng.randrange(len(specs))
        B = rng.choice([1, 1, 1, 2, 5, 17, 64])
        s = torch.from_numpy(sample(specs[gi][0], B, 1000 + i).syndromes).to("cuda:0")
        reqs.append((gi, s))
    alone = [graphs[gi].decode(s) for gi, s in reqs]
    torch.cuda.synchronize()
    srv = P.Server(graphs, slots=3, max_batch_requests=32, max_batch_shots=512)
    tickets = [None] * len(reqs)

    def producer():
        for i, (gi, s) in enumerate(reqs):
            tickets[i] = srv.submit(gi, s)
            time.sleep(rng.random() * 4e-4)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    lat = [srv.wait(t) for t, _ in tickets]
    info = srv.info()
    for (t, (c, o, st)), (c0, o0, st0) in zip(tickets, alone):
        assert torch.equal(c, c0) and torch.equal(o, o0) and torch.equal(st[:, DET], st0[:, DET])
    assert info["requests"] == len(reqs)
    assert 1 < info["batches"] < len(reqs)  # requests were batched
    assert min(lat) > 0.0
    # served outputs against the oracle: every graph's served shots, gathered
    # over its requests, sampled
    for gi, (dem, L, M, T) in enumerate(specs):
        idx = [i for i, (g, _) in enumerate(reqs) if g == gi]
        synd = np.concatenate([reqs[i][1].cpu().numpy() for i in idx])
        e = np.concatenate([P.unpack_bits(tickets[i][1][0], dem.n) for i in idx])
        st = np.concatenate([tickets[i][1][2].cpu().numpy() for i in idx])
        check_valid(dem, e, synd, st)
        print(sampled_oracle_parity(dem, graphs[gi], synd, e, st, 24, 900 + gi, f"served {dem.name}"), flush=True)
    srv.close()
    for G in graphs:
        G.close()


def test_server_rejects_oversized_request(torch_cuda):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem = code_capacity_dem(5, 0.05)
    G = P.Graph.from_dem(dem, permutations(dem.n, 8, 1), L=8, M=3, T_max=10)
    srv = P.Server([G], slots=1, max_batch_requests=4, max_batch_shots=16)
    s = torch.zeros((17, dem.m), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(P.VibeError):
        srv.submit(0, s)
    srv.close()
    G.close()


def test_admission_by_footprint(torch_cuda):
    """The pool is a budget smaller than the worst case: room for one batch
    of 4 shots of the d = 7 circuit graph.  A 64-shot request on that graph
    is refused at submission (its footprint exceeds the pool); 4-shot and
    1-shot requests are admitted, and a stream of them on two graphs is
    served with no batch larger than the pool allows, every output equal
    to the single-request decode, and the pool never over-committed."""
    import paper_2508_15743_amd as P

    torch = torch_cuda
    dem7, dem5 = circuit_dem(7, 7, 1e-3), code_capacity_dem(5, 0.05)
    G7 = P.Graph.from_dem(dem7, permutations(dem7.n, 32, 11), L=32, M=5, T_max=20)
    G5 = P.Graph.from_dem(dem5, permutations(dem5.n, 16, 12), L=16, M=5, T_max=32)
    probe = P.Server([G7], slots=1, max_batch_requests=8, max_batch_shots=4)
    budget = probe.info()["pool_bytes"]  # one full 4-shot batch of the d = 7 graph
    probe.close()
    srv = P.Server([G7, G5], slots=3, max_batch_requests=8, max_batch_shots=64, hbm_budget=budget)
    assert srv.info()["pool_bytes"] == budget
    big = torch.from_numpy(sample(dem7, 64, 13).syndromes).to("cuda:0")
    with pytest.raises(P.VibeError) as ei:
        srv.submit(0, big)
    assert ei.value.code == P.VIBE_ENOMEM
    reqs = [(0, big[:4].contiguous())]
    for i in range(40):
        gi = i % 2
        d = (dem7, dem5)[gi]
        reqs.append((gi, torch.from_numpy(sample(d, 1, 200 + i).syndromes).to("cuda:0")))
    alone = [(G7, G5)[gi].decode(s) for gi, s in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(gi, s) for gi, s in reqs]
    for t, _ in tickets:
        srv.wait(t)
    info = srv.info()
    for (t, (c, o, st)), (c0, o0, st0) in zip(tickets, alone):
        assert torch.equal(c, c0) and torch.equal(o, o0) and torch.equal(st[:, DET], st0[:, DET])
    assert info["requests"] == len(reqs)
    assert 0 < info["peak_bytes"] <= budget
    print(f"pool {budget / 2**20:.1f} MiB, peak in use {info['peak_bytes'] / 2**20:.1f} MiB, "
          f"{info['batches']} batches for {info['requests']} requests", flush=True)
    srv.close()
    G7.close()
    G5.close()
