"""GPU parity of the force-field options against the FP64 oracle: the CHARMM switch of
the Lennard-Jones term (r_on = 7.5 A for R = 9 A, the paper's benchmark setting) and
scaled 1-4 pairs (AMBER factors 1/2 and 1/1.2) read from the 1-4 bitmaps, in the forces,
energies, virials, per-atom energies, the adjoint and the Ewald corrections; both
precisions, the full- and half-shell cluster kernels."""

import numpy as np
import pytest

import nbtest_util as U
from oracle import oracle as O
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

FF = dict(lj_switch_on=7.5, scale14_lj=0.5, scale14_coul=1 / 1.2)
KERNELS = [H.NB_KERNEL_AUTO, "cluster8", "half8", "cluster4_static"]


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def chain14():
    return S.with_chain_14(U.small_chain())


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["chain14", "cfg2_14", "cfg1_switch"])
def test_switch_and_14_pairs_match_oracle(which, precision, kernel, chain14):
    if which == "chain14":
        s, ff = chain14, FF
    elif which == "cfg2_14":
        s, ff = S.with_chain_14(U.cached_config(2)), FF
    else:
        s, ff = U.cached_config(1), dict(lj_switch_on=7.5)
    _print_case("ff", which=which, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True, **ff)
    ref = U.oracle_for(s, precision, **ff)
    tol = 1e-12 if precision == H.NB_FP64 else 1e-5
    print(f"  rel_rms={U.rel_rms(out['force'], ref['force']):.3e} "
          f"max_rel_atom={U.max_rel_atom(out['force'], ref['force']):.3e}")
    U.assert_forces(out["force"], ref["force"], precision, tol)
    scale = np.abs(ref["energy"]).sum()
    assert abs(out["energy"][0] - ref["energy_total"]) <= (1e-12 if precision == H.NB_FP64 else 1e-6) * scale
    assert U.rel_rms(out["virial"][0], ref["virial"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert out["status"] == 0


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_adjoint_with_switch_and_14_pairs(precision, chain14):
    s = chain14
    out = U.gpu_eval(s, precision, backward=True, **FF)
    ref = U.oracle_for(s, precision, **FF)
    tol = 1e-11 if precision == H.NB_FP64 else 1e-5
    U.assert_forces(out["grad_pos"], -ref["force"], precision, tol)
    assert U.rel_rms(out["grad_charge"], ref["phi"]) <= tol
    lj = s.eps > 0
    np.testing.assert_allclose(out["grad_sigma"][lj], ref["dsigma"][lj], rtol=tol * 10, atol=tol)
    np.testing.assert_allclose(out["grad_eps"][lj], ref["deps"][lj], rtol=tol * 10, atol=tol)


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_ewald_corrections_of_14_pairs(precision, chain14):
    s = chain14
    out = U.gpu_eval(s, precision, **FF)
    b, p, ws = out["batch"], out["params"], out["ws"]
    force = torch.zeros((b.n_atoms, 3), dtype=torch.float64, device="cuda")
    energy = torch.zeros(1, dtype=torch.float64, device="cuda")
    vir = torch.zeros((1, 3, 3), dtype=torch.float64, device="cuda")
    H.ewald_corrections(b, p, ws, force, energy, vir)
    torch.cuda.synchronize()
    ref = O.ewald_corrections_system(U.rounded(s, precision), ke=H.COULOMB_K, scale14_coul=FF["scale14_coul"])
    np.testing.assert_allclose(force.cpu().numpy(), ref["force"], rtol=0, atol=1e-13 * np.abs(ref["force"]).max())
    assert abs(float(energy.cpu()[0]) - ref["energy_total"]) <= 1e-12 * (abs(ref["e_excl"]) + abs(ref["e_self"]))
    np.testing.assert_allclose(vir.cpu().numpy()[0], ref["virial"], rtol=0, atol=1e-12 * np.abs(ref["virial"]).max())


def test_batch_with_and_without_14_lists(chain14):
    systems = [chain14, U.cached_config(1), S.with_chain_14(S.solvated_chain(30.0, 80, 800, seed=4, cutoff=9.0,
                                                                                beta=0.34))]
    out = U.gpu_eval(systems, H.NB_MIXED, **FF)
    off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
    for k, s in enumerate(systems):
        ref = U.oracle_for(s, H.NB_MIXED, **FF)
        U.assert_forces(out["force"][off[k]:off[k + 1]], ref["force"], H.NB_MIXED, 1e-5)
        alone = U.gpu_eval(s, H.NB_MIXED, **FF)
        np.testing.assert_array_equal(out["force"][off[k]:off[k + 1]], alone["force"])


def test_far_14_pair_is_reported_and_left_unscaled(chain14):
    """1-4 pairs are held in the 64-index bitmaps only (as in the paper): a farther one
    sets NB_STATUS_FAR_PAIR14 and interacts as a plain pair."""
    s = chain14
    rows = [list(s.pair14_index[s.pair14_offset[i]:s.pair14_offset[i + 1]]) for i in range(s.n)]
    far = (0, 200)
    rows[far[0]].append(far[1])
    off = np.zeros(s.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    t = S.System(**{**s.__dict__})
    t.pair14_offset, t.pair14_index = off, np.array([j for r in rows for j in r], np.int32)
    out = U.gpu_eval(t, H.NB_FP64, **FF)
    assert out["status"] & H.NB_STATUS_FAR_PAIR14
    ref = U.oracle_for(s, H.NB_FP64, **FF)  # without the far pair in the 1-4 list
    U.assert_forces(out["force"], ref["force"], H.NB_FP64, 1e-12)
