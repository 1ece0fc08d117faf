"""GPU parity with excluded atoms that sit at the same point (a virtual site on its
parent atom, a hydrogen collapsed onto its oxygen), against the FP64 oracle.

An excluded pair takes no part in the real-space pair term (section 3: bonded partners
are left out through the exclusion bitmaps), so a pair at r = 0 must leave no trace in
the pair kernels, whose lanes evaluate every pair of a group and select the excluded
ones away: an infinite or undefined r^-12 or erfc(beta r)/r in such a lane may not reach
a sum.  The Ewald corrections do count such a pair, through the r -> 0 limit of
erf(beta r)/r, 2 beta / sqrt(pi), with no force.  The oracle pins that limit to the self
term on the CPU; here every kernel, both precisions, the adjoint, the force VJP and the
force-field variant are held to it."""

import numpy as np
import pytest

import nbtest_util as U
from oracle import oracle as O
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KERNELS = [H.NB_KERNEL_ATOM, H.NB_KERNEL_CLUSTER, "cluster8", "cluster4_static", "half8", "half4_dynamic"]
FF = dict(lj_switch_on=7.5, scale14_lj=0.5, scale14_coul=1 / 1.2)
TOL = {H.NB_FP64: 1e-12, H.NB_MIXED: 1e-5}
# pairs (i, j) of the 600-atom chain, j listed in the exclusion row of i; j is put on i
CHAIN_PAIRS = [(0, 1), (5, 6), (10, 12), (20, 21), (27, 29)]


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _collapse(s, pairs):
    t = S.System(**{**s.__dict__})
    t.pos = s.pos.copy()
    for i, j in pairs:
        assert j in s.excl_index[s.excl_offset[i]:s.excl_offset[i + 1]]
        t.pos[j] = t.pos[i]
    t.name = s.name + "_coincident"
    return t


def coincident(which):
    if which == "water":
        # the first hydrogen of each of the first 30 waters of the 648-atom box on its oxygen
        return _collapse(U.cached_config(1), [(3 * w, 3 * w + 1) for w in range(30)])
    if which == "chain":
        return _collapse(U.small_chain(), CHAIN_PAIRS)
    return _collapse(S.with_chain_14(U.small_chain()), CHAIN_PAIRS)


def _finite(out, keys):
    for k in keys:
        assert np.all(np.isfinite(out[k])), k


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["water", "chain"])
def test_forces_energy_virial_with_coincident_excluded_atoms(which, precision, kernel):
    s = coincident(which)
    _print_case("coincident-forces", which=which, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True)
    ref = U.oracle_for(s, precision)
    _finite(out, ("force", "energy", "virial", "atom_energy", "energy2"))
    tol = TOL[precision]
    U.assert_forces(out["force"], ref["force"], precision, tol)
    assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
    assert U.rel_rms(out["virial"][0], ref["virial"]) <= 10 * tol
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= 10 * tol
    assert out["status"] == 0


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster4_static", H.NB_KERNEL_ATOM])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["water", "chain"])
def test_adjoint_with_coincident_excluded_atoms(which, precision, kernel):
    s = coincident(which)
    _print_case("coincident-adjoint", which=which, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True)
    ref = U.oracle_for(s, precision)
    _finite(out, ("grad_pos", "grad_charge", "grad_sigma", "grad_eps"))
    tol = 1e-11 if precision == H.NB_FP64 else TOL[precision]
    U.assert_forces(out["grad_pos"], -ref["force"], precision, tol)
    assert U.rel_rms(out["grad_charge"], ref["phi"]) <= tol
    present = np.unique(s.type)
    lj = present[s.eps[present] > 0]
    np.testing.assert_allclose(out["grad_sigma"][lj], ref["dsigma"][lj], rtol=tol * 10, atol=tol)
    np.testing.assert_allclose(out["grad_eps"][lj], ref["deps"][lj], rtol=tol * 10, atol=tol)
    assert out["status"] == 0


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster8", "half8"])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_switch_and_14_pairs_with_coincident_excluded_atoms(precision, kernel):
    s = coincident("chain14")
    _print_case("coincident-ff", precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True, **FF)
    ref = U.oracle_for(s, precision, **FF)
    _finite(out, ("force", "energy", "virial", "atom_energy"))
    tol = TOL[precision]
    U.assert_forces(out["force"], ref["force"], precision, tol)
    assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= 10 * tol
    assert out["status"] == 0


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_force_vjp_with_coincident_excluded_atoms(precision):
    s = coincident("chain")
    _print_case("coincident-vjp", precision=precision, n=s.n)
    out = U.gpu_eval(s, precision)
    b, p, ws = out["batch"], out["params"], out["ws"]
    T = b.sigma.shape[0]
    v = np.random.default_rng(3).standard_normal((s.n, 3))
    vd = torch.as_tensor(v, dtype=torch.float64, device="cuda").contiguous()
    gq = torch.full((b.n_atoms,), np.nan, dtype=torch.float64, device="cuda")
    gs = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    ge = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    H.nonbonded_force_vjp(b, p, ws, vd, gq, gs, ge)
    torch.cuda.synchronize()
    ref = U.oracle_for(s, precision, vjp=v)
    tol = 1e-11 if precision == H.NB_FP64 else 2e-5
    got_q, got_s, got_e = gq.cpu().numpy(), gs.cpu().numpy(), ge.cpu().numpy()
    assert np.all(np.isfinite(got_q)) and np.all(np.isfinite(got_s)) and np.all(np.isfinite(got_e))
    assert U.rel_rms(got_q, ref["vjp_charge"]) <= tol
    lj = s.eps > 0
    np.testing.assert_allclose(got_s[lj], ref["vjp_sigma"][lj], rtol=tol * 10,
                               atol=tol * np.abs(ref["vjp_sigma"][lj]).max())
    np.testing.assert_allclose(got_e[lj], ref["vjp_eps"][lj], rtol=tol * 10,
                               atol=tol * np.abs(ref["vjp_eps"][lj]).max())
    assert H.read_status(ws) == 0


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["water", "chain"])
def test_ewald_corrections_take_the_zero_distance_limit(which, precision):
    """The corrections of a pair at r = 0: energy -k_e q_i q_j 2 beta / sqrt(pi), no force."""
    s = coincident(which)
    _print_case("coincident-ewald", which=which, precision=precision, n=s.n)
    out = U.gpu_eval(s, precision)
    b, p, ws = out["batch"], out["params"], out["ws"]
    force = torch.full((b.n_atoms, 3), 7.0, dtype=torch.float64, device="cuda")
    energy = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    vir = torch.full((1, 3, 3), 7.0, dtype=torch.float64, device="cuda")
    H.ewald_corrections(b, p, ws, force, energy, vir)
    torch.cuda.synchronize()
    f, e, w = force.cpu().numpy(), energy.cpu().numpy(), vir.cpu().numpy()
    ref = O.ewald_corrections_system(U.rounded(s, precision), ke=H.COULOMB_K)
    assert np.all(np.isfinite(f)) and np.isfinite(e[0]) and np.all(np.isfinite(w))
    assert U.rel_rms(f, ref["force"]) <= 1e-13
    assert abs(e[0] - ref["energy_total"]) <= 1e-12 * (abs(ref["e_excl"]) + abs(ref["e_self"]))
    assert U.rel_rms(w[0], ref["virial"]) <= 1e-12
    assert H.read_status(ws) == 0


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster4_static"])
@pytest.mark.parametrize("table,tol,max_rel", [(1, 1e-4, 1e-3), (2, 1e-5, 1e-4)])
def test_tables_with_coincident_excluded_atoms(table, tol, max_rel, kernel):
    """At r = 0 the table index comes from an undefined r; it is clamped to the table and
    the lane's terms are selected away."""
    s = coincident("water")
    _print_case("coincident-tables", table=table, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, H.NB_MIXED, kernel=kernel, energy_call=True, table=table)
    ref = U.oracle_for(s, H.NB_MIXED)
    _finite(out, ("force", "energy", "virial", "atom_energy"))
    assert U.rel_rms(out["force"], ref["force"]) <= tol
    assert U.max_rel_atom(out["force"], ref["force"]) <= max_rel
    assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
    assert out["status"] == 0
