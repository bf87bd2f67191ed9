"""The C ABI library: it loads and exports every function the header
declares.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vibelsd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vibe_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("vibe_graph_create", "vibe_graph_destroy", "vibe_graph_info", "vibe_decode",
              "vibe_decode_plain", "vibe_bp_ensemble", "vibe_lsd", "vibe_last_error",
              "vibe_version"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2508_15743_amd as P

    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libvibelsd.so not built")
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert P.vibe_version().startswith("vibelsd")
    assert set(P.EXPORTS) == set(declared_functions())


def test_library_is_gfx950():
    import paper_2508_15743_amd as P

    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libvibelsd.so not built")
    blob = open(P.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_graph_create_needs_a_gpu():
    import torch

    import paper_2508_15743_amd as P
    from synth.dem import code_capacity_dem
    from synth.sample import permutations

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    dem = code_capacity_dem(3, 0.1)
    with pytest.raises(RuntimeError):
        P.Graph.from_dem(dem, permutations(dem.n, 4, 0), L=4, M=2, T_max=5)
