"""GPU check of the allocation-free entry point (nb_nonbonded_forces_noalloc): its forces,
energies and virials equal those of nb_build_cells + nb_nonbonded_forces on a caller's
workspace, bit for bit (the same kernels on the same inputs), on two calls in a row, the
second with a smaller input, in both precisions."""

import numpy as np
import pytest

import nbtest_util as U
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _noalloc(systems, precision):
    dt = torch.float64 if precision == H.NB_FP64 else torch.float32
    b = H.device_batch(systems, dtype=dt)
    p = H.make_params(systems[0].cutoff, systems[0].beta, precision)
    force = torch.full((b.n_atoms, 3), 7.0, dtype=torch.float64, device="cuda")
    energy = torch.full((b.n_systems,), 7.0, dtype=torch.float64, device="cuda")
    vir = torch.full((b.n_systems, 3, 3), 7.0, dtype=torch.float64, device="cuda")
    H.nonbonded_forces_noalloc(b, p, force, energy, vir)
    torch.cuda.synchronize()
    return force.cpu().numpy(), energy.cpu().numpy(), vir.cpu().numpy()


@pytest.mark.parametrize("precision", [H.NB_MIXED, H.NB_FP64])
def test_noalloc_equals_the_workspace_entry_points(precision):
    big = [U.small_chain(), S.water_box(1500, 26.0, seed=3)]
    small = [U.cached_config(1)]
    for systems in (big, small):  # the second call is smaller than the first
        print(f"[case] noalloc precision={precision} atoms={sum(s.n for s in systems)}", flush=True)
        f, e, v = _noalloc(systems, precision)
        ref = U.gpu_eval(systems, precision)
        np.testing.assert_array_equal(f, ref["force"])
        np.testing.assert_array_equal(e, ref["energy"])
        np.testing.assert_array_equal(v, ref["virial"])
        # and against the oracle, as every other forces call
        off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
        for k, s in enumerate(systems):
            o = U.oracle_for(s, precision)
            U.assert_forces(f[off[k]:off[k + 1]], o["force"], precision, 1e-12 if precision == H.NB_FP64 else 1e-5)
