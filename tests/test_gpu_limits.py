"""GPU parity at the edges of the accepted inputs, against the FP64 oracle:

* the largest type count the library accepts (NB_MAX_TYPES = 64) and a single type,
  forces and the per-type gradients of the adjoint;
* a cutoff just below half the box (the largest the minimum image allows, section 3);
* a system without charges (Lennard-Jones only) and one without Lennard-Jones
  (Ewald real-space Coulomb only).
"""

import numpy as np
import pytest

import nbtest_util as U
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KERNELS = [H.NB_KERNEL_AUTO, H.NB_KERNEL_CLUSTER, "cluster4_static", "half4_dynamic", H.NB_KERNEL_ATOM]
TOL = {H.NB_FP64: 1e-12, H.NB_MIXED: 1e-5}


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _types(s, T, seed):
    """The system with T Lennard-Jones types drawn for its atoms (every type used when
    the system has at least T atoms)."""
    rng = np.random.default_rng(seed)
    t = S.System(**{**s.__dict__})
    t.sigma = rng.uniform(2.5, 3.8, T)
    t.eps = rng.uniform(0.1, 0.9, T)
    t.type = (np.arange(s.n) % T).astype(np.int32)
    rng.shuffle(t.type)
    return t


def _check_forces(out, ref, precision):
    tol = TOL[precision]
    U.assert_forces(out["force"], ref["force"], precision, tol)
    assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
    assert out["status"] == 0


def _check_adjoint(out, ref, s, precision):
    tol = 1e-11 if precision == H.NB_FP64 else TOL[precision]
    U.assert_forces(out["grad_pos"], -ref["force"], precision, tol)
    assert U.rel_rms(out["grad_charge"], ref["phi"]) <= tol
    lj = np.unique(s.type)
    lj = lj[s.eps[lj] > 0]
    np.testing.assert_allclose(out["grad_sigma"][lj], ref["dsigma"][lj], rtol=max(tol * 10, 1e-10), atol=tol)
    np.testing.assert_allclose(out["grad_eps"][lj], ref["deps"][lj], rtol=max(tol * 10, 1e-10), atol=tol)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("T", [1, H.NB_MAX_TYPES])
def test_one_type_and_the_most_types(T, precision, kernel):
    s = _types(U.small_chain(), T, seed=T)
    _print_case("types", T=T, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True)
    ref = U.oracle_for(s, precision)
    assert out["grad_sigma"].shape == (T,) and out["grad_eps"].shape == (T,)
    _check_forces(out, ref, precision)
    _check_adjoint(out, ref, s, precision)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_cutoff_just_below_half_the_box(precision, kernel):
    s = U.lattice_system((20.0, 20.0, 20.0), 2.4, seed=41, cutoff=9.99, beta=0.3)
    _print_case("half-box-cutoff", precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True)
    ref = U.oracle_for(s, precision)
    _check_forces(out, ref, precision)
    _check_adjoint(out, ref, s, precision)


def _lj_force_magnitude_sums(s):
    """Per atom, the sum over its in-range, non-excluded partners of the magnitudes of the
    two parts of the Lennard-Jones pair force, 24 eps (2 (sigma/r)^12 + (sigma/r)^6) / r
    with the Lorentz-Berthelot rule: the scale that single-precision pair terms are rounded
    on (near the potential's minimum the two parts cancel within one pair too)."""
    out = np.zeros(s.n)
    for i in range(s.n):
        d = s.pos[i] - s.pos
        d -= s.box * np.rint(d / s.box)
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        r2[s.excl_index[s.excl_offset[i]:s.excl_offset[i + 1]]] = np.inf
        m = r2 < s.cutoff ** 2
        sig = 0.5 * (s.sigma[s.type[i]] + s.sigma[s.type[m]])
        eps = np.sqrt(s.eps[s.type[i]] * s.eps[s.type[m]])
        sr6 = (sig * sig / r2[m]) ** 3
        out[i] = (24.0 * eps * (2.0 * sr6 * sr6 + sr6) / np.sqrt(r2[m])).sum()
    return out


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster4_static", H.NB_KERNEL_ATOM])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["no_charges", "no_lj"])
def test_lennard_jones_only_and_coulomb_only(which, precision, kernel):
    c = U.small_chain()
    s = S.System(**{**c.__dict__})
    if which == "no_charges":
        s.charge = np.zeros_like(c.charge)
    else:
        s.eps = np.zeros_like(c.eps)
    _print_case("one-term", which=which, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True)
    ref = U.oracle_for(s, precision)
    tol = 1e-11 if precision == H.NB_FP64 else TOL[precision]
    if which == "no_charges" and precision == H.NB_MIXED:
        # Without the Coulomb term some atoms' net force is the remainder of pair forces a
        # thousand times larger (|F| = 0.32 against 444 kJ/mol/A of |f_ij| summed for one
        # of them), so the per-atom error is bounded by the single-precision terms'
        # relative error times the sum of the terms, not by |F_i|.  The repulsive term
        # c12 r^-14 is r^-2 (from the fixed-point difference, r^2 and rsqrt: about 5 units
        # in the last place) to the 7th power: about 35 ulp = 2e-6 at worst (measured 9e-7).
        scale = _lj_force_magnitude_sums(s)
        for f in (out["force"], -out["grad_pos"]):
            assert U.rel_rms(f, ref["force"]) <= TOL[precision]
            err = np.linalg.norm(f - ref["force"], axis=1)
            worst = float((err[scale > 0] / scale[scale > 0]).max())
            print(f"  max |dF_i| / sum of term magnitudes = {worst:.3e}")
            assert np.all(err[scale == 0] == 0.0)
            assert worst <= 2e-6
        assert abs(out["energy"][0] - ref["energy_total"]) <= TOL[precision] * np.abs(ref["energy"]).sum()
        assert out["status"] == 0
    else:
        _check_forces(out, ref, precision)
        U.assert_forces(out["grad_pos"], -ref["force"], precision, tol)
    if which == "no_lj":
        assert not out["grad_eps"].any()
    # dE/dq_i = phi_i: zero when no atom is charged, the Coulomb term alone otherwise
    assert U.rel_rms(out["grad_charge"], ref["phi"]) <= tol
