"""GPU parity of the tabulated variant (nb_params.table) against the FP64 oracle: the
paper's linear tables (4096 intervals) within its 1e-4 relative force error, the cubic
Hermite tables (1024 intervals) within the direct evaluation's 1e-5; full- and half-shell
kernels, 8- and 4-atom clusters."""

import numpy as np
import pytest

import nbtest_util as U
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster8", "cluster4_static"])
@pytest.mark.parametrize("table,tol,max_rel", [(1, 1e-4, 1e-3), (2, 1e-5, 1e-4)])
@pytest.mark.parametrize("which", ["chain", "cfg2", "cfg5_rows"])
def test_tables_match_oracle(which, table, tol, max_rel, kernel):
    s = {"chain": U.small_chain, "cfg2": lambda: U.cached_config(2), "cfg5_rows": lambda: U.cached_config(5)}[which]()
    print(f"[case] tables which={which} table={table} kernel={kernel} n={s.n}", flush=True)
    out = U.gpu_eval(s, H.NB_MIXED, kernel=kernel, energy_call=True, table=table)
    rows = np.random.default_rng(3).choice(s.n, 256, replace=False) if which == "cfg5_rows" else None
    ref = U.oracle_for(s, H.NB_MIXED, rows=rows)
    f = out["force"] if rows is None else out["force"][rows]
    err, mx = U.rel_rms(f, ref["force"]), U.max_rel_atom(f, ref["force"])
    print(f"  rel_rms={err:.3e} max_rel_atom={mx:.3e}")
    assert err <= tol and mx <= max_rel
    if rows is None:
        assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
        assert U.rel_rms(out["virial"][0], ref["virial"]) <= tol
        assert U.rel_rms(out["atom_energy"], ref["energy"]) <= tol
    assert out["status"] == 0


def test_table_is_refused_with_the_switch_and_the_fp64_path_ignores_it():
    s = U.small_chain()
    b = H.device_batch([s])
    with pytest.raises(H.NbError):
        H.workspace_bytes(b, H.make_params(9.0, 0.34, table=1, lj_switch_on=7.5))
    a = U.gpu_eval(s, H.NB_FP64, table=1)
    c = U.gpu_eval(s, H.NB_FP64)
    np.testing.assert_array_equal(a["force"], c["force"])
