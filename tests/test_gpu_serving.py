"""Serving with continuous batching (through the C ABI).

Requests on several resident graphs are submitted from another thread at
irregular times while earlier batches are on the GPU.  Each request's outputs
must equal the single-request decode of the same syndromes bit for bit, and
the server must have formed batches of several requests.
"""
import random
import threading
import time

import numpy as np
import pytest

from synth.dem import circuit_dem, code_capacity_dem, phenomenological_dem
from synth.sample import permutations, sample

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
    with pytest.raises(P.VibeError):
        P.Server([G], slots=2, max_batch_requests=4, max_batch_shots=16, hbm_budget=1024)
    srv.close()
    G.close()
