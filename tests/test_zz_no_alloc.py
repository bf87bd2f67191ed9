"""vibe_decode_noalloc (the decode for callers that cannot allocate) against
vibe_decode on the same syndromes, through the C ABI: two calls in a row on
one graph, the second with a smaller batch, each equal to vibe_decode's
outputs bit for bit (corrections, observables, and every stats field but
the timing-dependent n_conv and member_iters).  The d = 9 circuit graph
needs more than one chunk of shots in the static array at the first
batch size and a BP grid cut to fit it; the code-capacity graph keeps its
message slab in LDS."""
import numpy as np
import pytest

from synth.dem import circuit_dem, code_capacity_dem
from synth.sample import permutations, sample

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


def _outs(torch, G, B):
    dev = "cuda:0"
    return (torch.full((B, G.words), -1, dtype=torch.int64, device=dev),
            torch.full((B, max(G.k, 1)), 7, dtype=torch.uint8, device=dev),
            torch.full((B, 8), -1, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("which", ["code_capacity_d5", "circuit_d9"])
def test_noalloc_equals_decode(torch_cuda, which):
    import paper_2508_15743_amd as P

    torch = torch_cuda
    if which == "circuit_d9":
        dem, L, M, T, sizes = circuit_dem(9, 9, 1e-3), 32, 5, 20, (1500, 300)
    else:
        dem, L, M, T, sizes = code_capacity_dem(5, 0.05), 16, 5, 32, (6000, 1000)
    G = P.Graph.from_dem(dem, permutations(dem.n, L, 71), L=L, M=M, T_max=T)
    synd = torch.from_numpy(sample(dem, sizes[0], 72).syndromes).to("cuda:0")
    for B in sizes:
        s = synd[:B].contiguous()
        ref = G.decode(s, out=_outs(torch, G, B))
        got = _outs(torch, G, B)
        print(f"{which}: vibe_decode_noalloc on {B} shots", flush=True)
        P.vibe_decode_noalloc(G.handle, s, B, got[0], got[1], got[2], None)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]), which
        assert torch.equal(got[1], ref[1]), which
        assert torch.equal(got[2][:, DET], ref[2][:, DET]), which
        assert ((got[2][:, 0].cpu().numpy() & 3) != 0).all()
    # B = 0 does nothing; a NULL output is refused with nothing written
    P.vibe_decode_noalloc(G.handle, synd, 0, None, None, None, None)
    out = _outs(torch, G, 4)
    with pytest.raises(P.VibeError) as ei:
        P.vibe_decode_noalloc(G.handle, synd[:4], 4, None, out[1], out[2], None)
    assert ei.value.code == P.VIBE_EINVAL
    torch.cuda.synchronize()
    assert (out[1] == 7).all() and (out[2] == -1).all()
    G.close()
