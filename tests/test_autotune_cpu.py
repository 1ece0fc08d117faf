"""Host logic of the autotuner: workload signatures, the JSON cache and the candidate
space (every candidate must pass the library's host validation)."""

import ctypes

import numpy as np
import pytest

from paper_0902_0827_amd import autotune as A
from paper_0902_0827_amd import nbhip as H
from test_abi_cpu import fake_system, ws_bytes


class _FakeBatch:
    def __init__(self, n, B, box, T=10):
        self.n_atoms, self.n_systems = n, B
        self.box = np.asarray(box, dtype=np.float64)
        self.sigma = np.zeros(T)


def test_signature_separates_what_matters_and_ignores_noise():
    a = _FakeBatch(23600, 1, [[60.0, 60.0, 60.0]])
    base = A.signature(a, 9.0, 0.34, H.NB_MIXED, "gpu")
    assert A.signature(_FakeBatch(23601, 1, [[60.0, 60.0, 60.0]]), 9.0, 0.34, H.NB_MIXED, "gpu") == base
    for other in (A.signature(a, 12.0, 0.34, H.NB_MIXED, "gpu"), A.signature(a, 9.0, 0.26, H.NB_MIXED, "gpu"),
                  A.signature(a, 9.0, 0.34, H.NB_FP64, "gpu"), A.signature(a, 9.0, 0.34, H.NB_MIXED, "other"),
                  A.signature(_FakeBatch(47200, 1, [[75.6, 75.6, 75.6]]), 9.0, 0.34, H.NB_MIXED, "gpu"),
                  A.signature(_FakeBatch(23600, 2, [[60.0] * 3, [60.0] * 3]), 9.0, 0.34, H.NB_MIXED, "gpu")):
        assert other != base


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "tune.json"))
    assert A.load_cache() == {}
    entry = {"params": {"kernel": 2, "cluster_size": 8, "cell_div_xy": 2, "cell_div_z": 8, "split": 1,
                        "schedule": 1, "wg_per_cu": 0}, "sec": 1e-4}
    A.store_cache("k1", entry)
    A.store_cache("k2", dict(entry, sec=2e-4))
    data = A.load_cache()
    assert set(data) == {"k1", "k2"} and data["k1"]["sec"] == 1e-4
    p = A.params_from(data["k1"]["params"], 9.0, 0.34, H.NB_MIXED)
    assert (p.kernel, p.cluster_size, p.cell_div_z, p.schedule) == (2, 8, 8, 1)
    (tmp_path / "tune.json").write_text("not json")
    assert A.load_cache() == {}  # a damaged cache is ignored, not fatal


@pytest.mark.parametrize("precision", [H.NB_MIXED, H.NB_FP64])
def test_every_candidate_passes_host_validation(precision):
    s = fake_system((23600,), L=60.0)
    best = {k: 0 for k in A.PARAM_KEYS}
    n = 0
    for stage in range(3):
        for over in A.stage_candidates(stage, best, precision):
            p = A.params_from(dict(best, **over), 9.0, 0.34, precision)
            code, nbytes = ws_bytes(s, p)
            assert code == H.NB_OK, (over, H.last_error())
            assert nbytes > 0
            n += 1
    assert n >= 10
