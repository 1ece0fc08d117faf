"""GPU parity on box shapes and positions that take the less common paths of the build
and of the pair kernels' neighbour windows, against the FP64 oracle (section 3: the
minimum image in a periodic box, the cell list whose stencil covers the cutoff):

* an elongated box, whose stencil spans the whole box in x and y but not in z, and a
  slab, whose stencil spans it in z only: the column windows then take whole columns in
  one case and wrap in z in the other;
* atoms exactly on the box's faces (x = 0 and x = L, the same point of the periodic box),
  and their fixed-point cells, bit for bit.
"""

import numpy as np
import pytest

import nbtest_util as U
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KERNELS = [H.NB_KERNEL_ATOM, H.NB_KERNEL_CLUSTER, "cluster8", "cluster4_static", "half8", "half4_dynamic"]
TOL = {H.NB_FP64: 1e-12, H.NB_MIXED: 1e-5}
SHAPES = {"elongated": (18.5, 19.0, 90.0), "slab": (90.0, 88.0, 18.5)}


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _check(out, ref, precision):
    tol = TOL[precision]
    U.assert_forces(out["force"], ref["force"], precision, tol)
    scale = float(np.abs(ref["energy"]).sum())
    assert abs(out["energy"][0] - ref["energy_total"]) <= tol * scale
    assert U.rel_rms(out["virial"][0], ref["virial"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert out["status"] == 0


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("shape", ["elongated", "slab"])
def test_elongated_and_slab_boxes(shape, precision, kernel):
    s = U.lattice_system(SHAPES[shape], 2.6, seed=31)
    _print_case("shape", shape=shape, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True)
    ref = U.oracle_for(s, precision)
    print(f"  rel_rms={U.rel_rms(out['force'], ref['force']):.3e}")
    _check(out, ref, precision)


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("shape", ["elongated", "slab"])
def test_binning_of_elongated_and_slab_boxes(shape, precision):
    s = U.lattice_system(SHAPES[shape], 2.6, seed=31)
    _print_case("shape-binning", shape=shape, precision=precision)
    out = U.gpu_eval(s, precision, cell_div_xy=2, cell_div_z=8)
    ws = U.workspace_arrays(out)
    ref = U.oracle_binning([s], precision, (2, 2, 8))
    np.testing.assert_array_equal(ws["cell_start"], ref["cell_start"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, 3], ref["order"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, :3], ref["sorted_fixed"])


def on_faces(s):
    """The system translated so that atom 0 lies on x = 0, atom 1 on y = 0 and atom 2 on
    z = 0 exactly; then atom 0 is moved by one box length to x = L, the same point of the
    periodic box.  Translation leaves every pair distance unchanged."""
    t = S.System(**{**s.__dict__})
    pos = s.pos - np.array([s.pos[0, 0], s.pos[1, 1], s.pos[2, 2]])
    pos[0, 0] += s.box[0]
    assert pos[0, 0] == s.box[0] and pos[1, 1] == 0.0 and pos[2, 2] == 0.0
    t.pos = pos
    return t


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster4_static", H.NB_KERNEL_ATOM])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_atoms_exactly_on_the_box_faces(precision, kernel):
    s = on_faces(U.small_chain())
    _print_case("faces", precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True, cell_div_xy=2, cell_div_z=8)
    ref = U.oracle_for(s, precision)
    _check(out, ref, precision)
    ws = U.workspace_arrays(out)
    rb = U.oracle_binning([s], precision, (2, 2, 8))
    np.testing.assert_array_equal(ws["cell_start"], rb["cell_start"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, 3], rb["order"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, :3], rb["sorted_fixed"])
    if precision == H.NB_FP64:
        # x = L is the face x = 0 of the periodic box: fixed-point coordinate 0 (single
        # precision rounds L itself, so only the comparison with the oracle above applies)
        where = {int(o): k for k, o in enumerate(ws["sorted_fixed"][:, 3])}
        assert ws["sorted_fixed"][where[0], 0] == 0
        assert ws["sorted_fixed"][where[1], 1] == 0 and ws["sorted_fixed"][where[2], 2] == 0


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("shape", ["elongated", "slab"])
def test_adjoint_and_force_vjp_on_elongated_and_slab_boxes(shape, precision):
    s = U.lattice_system(SHAPES[shape], 2.6, seed=31)
    _print_case("shape-gradients", shape=shape, precision=precision, n=s.n)
    out = U.gpu_eval(s, precision, backward=True)
    v = np.random.default_rng(13).standard_normal((s.n, 3))
    ref = U.oracle_for(s, precision, vjp=v)
    tol = 1e-11 if precision == H.NB_FP64 else TOL[precision]
    U.assert_forces(out["grad_pos"], -ref["force"], precision, tol)
    assert U.rel_rms(out["grad_charge"], ref["phi"]) <= tol
    np.testing.assert_allclose(out["grad_sigma"], ref["dsigma"], rtol=tol * 10, atol=tol)
    np.testing.assert_allclose(out["grad_eps"], ref["deps"], rtol=tol * 10, atol=tol)
    b, p, ws = out["batch"], out["params"], out["ws"]
    T = b.sigma.shape[0]
    vd = torch.as_tensor(v, dtype=torch.float64, device="cuda").contiguous()
    gq = torch.full((b.n_atoms,), np.nan, dtype=torch.float64, device="cuda")
    gs = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    ge = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    H.nonbonded_force_vjp(b, p, ws, vd, gq, gs, ge)
    torch.cuda.synchronize()
    vtol = 1e-11 if precision == H.NB_FP64 else 2e-5
    assert U.rel_rms(gq.cpu().numpy(), ref["vjp_charge"]) <= vtol
    np.testing.assert_allclose(gs.cpu().numpy(), ref["vjp_sigma"], rtol=vtol * 10,
                               atol=vtol * np.abs(ref["vjp_sigma"]).max())
    np.testing.assert_allclose(ge.cpu().numpy(), ref["vjp_eps"], rtol=vtol * 10,
                               atol=vtol * np.abs(ref["vjp_eps"]).max())
    assert H.read_status(ws) == 0
