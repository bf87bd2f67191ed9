"""The stored oracle results (tests/golden/oracle_*.npz, written by
oracle/fixtures.py) still describe the current inputs and the current
oracle: the input digests match freshly generated inputs, and a sample of
shots decoded again by the oracle gives the stored corrections, flags and
witnesses.  CPU only."""
import os

import numpy as np
import pytest

from oracle import fixtures as F
from oracle import oracle as O

NT = min(8, os.cpu_count() or 1)


@pytest.mark.parametrize("name,sample", [("phenom_d11", 96), ("circuit_d9", 3)])
def test_fixture_matches_inputs_and_oracle(name, sample):
    path = F.path_for(name)
    assert os.path.exists(path), f"run python -m oracle.fixtures {name}"
    ref = F.load(name)
    meta = ref["meta"]
    dem, perms, b, n = F.workload_inputs(name, meta["shots"])
    assert meta["syndromes_sha"] == F.array_digest(b.syndromes[:n])
    assert meta["perms_sha"] == F.array_digest(perms)
    assert len(ref["ehat_digest"]) == n == meta["shots"]
    w = F.WORKLOADS[name]
    assert (meta["L"], meta["M"], meta["T"], meta["lsd_order"]) == (w["L"], w["M"], w["T"], w["lsd_order"])
    # a spread sample, including LSD shots
    rng = np.random.default_rng(5)
    lsd = np.flatnonzero(ref["flags"] & 2)
    pick = np.unique(np.concatenate([rng.choice(n, sample - sample // 2, replace=False),
                                     rng.choice(lsd, sample // 2, replace=False)]))
    r = O.decode(O.OracleGraph(dem), perms, b.syndromes[pick], L=w["L"], M=w["M"], T=w["T"],
                 alpha=w["alpha"], threads=NT, lsd_order=w["lsd_order"])
    assert np.array_equal(F.ehat_digest(r["ehat"]), ref["ehat_digest"][pick])
    assert np.array_equal(r["rec"][:, 0].astype(np.uint8), ref["flags"][pick])
    assert np.array_equal(r["obs"], ref["obs"][pick])
    np.testing.assert_array_equal(r["min_q_gap"], ref["min_q_gap"][pick])
    np.testing.assert_array_equal(r["min_abs_post"], ref["min_abs_post"][pick])
    # the stored set bits (circuit workload) are those of the digests
    if "ehat_indptr" in ref:
        ip, ix = ref["ehat_indptr"], ref["ehat_indices"]
        for j, i in enumerate(pick):
            assert np.flatnonzero(r["ehat"][j]).tolist() == ix[ip[i]:ip[i + 1]].tolist()
