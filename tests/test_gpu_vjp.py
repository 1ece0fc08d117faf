"""GPU parity of the force VJP (the double backward of force matching) against the FP64
oracle: with L = sum_i v_i . F_i, the derivatives dL/dq_i, dL/dsigma_t and dL/deps_t of
the real-space pair forces, with and without the force-field options (switch, scaled
1-4 pairs), both precisions, the cluster kernels (the VJP always runs full shell), one
and several items per cluster, and a batch of systems sharing the type table.  The
oracle's VJP is pinned to finite differences of its own forces on the CPU."""

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
# the mixed path sums FP32 pair terms in double: relative RMS of the per-atom dL/dq and
# the relative error of the per-type sums
TOL = {H.NB_FP64: 1e-11, H.NB_MIXED: 2e-5}


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _v(n, seed):
    return np.random.default_rng(seed).standard_normal((n, 3))


def _gpu_vjp(systems, precision, v, kernel=H.NB_KERNEL_AUTO, **ff):
    out = U.gpu_eval(systems, precision, kernel=kernel, **ff)
    b, p, ws = out["batch"], out["params"], out["ws"]
    T = b.sigma.shape[0]
    vd = torch.as_tensor(v, dtype=torch.float64, device="cuda").contiguous()
    gq = torch.full((b.n_atoms,), np.nan, dtype=torch.float64, device="cuda")
    gs = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    ge = torch.full((T,), np.nan, dtype=torch.float64, device="cuda")
    H.nonbonded_force_vjp(b, p, ws, vd, gq, gs, ge)
    torch.cuda.synchronize()
    return dict(q=gq.cpu().numpy(), sigma=gs.cpu().numpy(), eps=ge.cpu().numpy(), status=H.read_status(ws))


def _check(got, ref_q, ref_s, ref_e, eps, precision):
    tol = TOL[precision]
    assert U.rel_rms(got["q"], ref_q) <= tol, U.rel_rms(got["q"], ref_q)
    lj = eps > 0
    scale = np.abs(ref_s[lj]).max()
    np.testing.assert_allclose(got["sigma"][lj], ref_s[lj], rtol=tol * 10, atol=tol * scale)
    scale = np.abs(ref_e[lj]).max()
    np.testing.assert_allclose(got["eps"][lj], ref_e[lj], rtol=tol * 10, atol=tol * scale)
    assert np.all(got["eps"][~lj] == 0.0)
    assert got["status"] == 0


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_AUTO, "cluster8", "half8", "cluster4_static"])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("ff", [False, True])
def test_force_vjp_matches_oracle(ff, precision, kernel):
    s = S.with_chain_14(U.small_chain()) if ff else U.small_chain()
    opts = FF if ff else {}
    _print_case("vjp", ff=ff, precision=precision, kernel=kernel, n=s.n)
    v = _v(s.n, 5)
    got = _gpu_vjp(s, precision, v, kernel=kernel, **opts)
    ref = U.oracle_for(s, precision, vjp=v, **opts)
    _check(got, ref["vjp_charge"], ref["vjp_sigma"], ref["vjp_eps"], s.eps, precision)


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_force_vjp_on_the_water_box(precision):
    """23,558-atom water box (many tiles, every cluster full): dL/dq on all atoms, per-type sums."""
    s = U.cached_config(2)
    _print_case("vjp_cfg2", precision=precision, n=s.n)
    v = _v(s.n, 9)
    got = _gpu_vjp(s, precision, v)
    ref = U.oracle_for(s, precision, vjp=v)
    _check(got, ref["vjp_charge"], ref["vjp_sigma"], ref["vjp_eps"], s.eps, precision)


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_force_vjp_over_a_batch(precision):
    """Three systems of different sizes in one call: dL/dq per atom, and the per-type sums
    taken over all of them (L sums over every system)."""
    systems = [U.small_chain(), S.config1(), S.solvated_chain(20.0, 20, 200, seed=4, cutoff=9.0, beta=0.34)]
    _print_case("vjp_batch", precision=precision, n=sum(x.n for x in systems))
    v = _v(sum(x.n for x in systems), 13)
    got = _gpu_vjp(systems, precision, v)
    off = np.cumsum([0] + [x.n for x in systems])
    refs = [U.oracle_for(x, precision, vjp=v[off[k]:off[k + 1]]) for k, x in enumerate(systems)]
    ref_q = np.concatenate([r["vjp_charge"] for r in refs])
    ref_s = sum(r["vjp_sigma"] for r in refs)
    # dL/deps_t = (sum over systems of the eps-scaled sums) / eps_t: the per-system values add
    ref_e = sum(r["vjp_eps"] for r in refs)
    _check(got, ref_q, ref_s, ref_e, systems[0].eps, precision)


def test_forces_autograd_uses_the_vjp():
    """NonbondedForces: backward through a force-matching loss gives the VJP with
    v = dLoss/dF, and refuses the position derivative."""
    s = U.small_chain()
    b = H.device_batch([s], dtype=torch.float64)
    p = H.make_params(s.cutoff, s.beta, H.NB_FP64)
    q = b.charge.clone().requires_grad_(True)
    sig = b.sigma.clone().requires_grad_(True)
    eps = b.eps.clone().requires_grad_(True)
    f = H.nonbonded_forces_autograd(b.pos, q, sig, eps, b, p)
    target = torch.zeros_like(f)
    loss = 0.5 * ((f - target) ** 2).sum()
    loss.backward()
    v = f.detach().cpu().numpy()  # dLoss/dF
    ref = O.evaluate_system(s, ke=H.COULOMB_K, vjp=v)
    assert U.rel_rms(q.grad.cpu().numpy(), ref["vjp_charge"]) <= 1e-11
    lj = s.eps > 0
    np.testing.assert_allclose(sig.grad.cpu().numpy()[lj], ref["vjp_sigma"][lj], rtol=1e-10)
    np.testing.assert_allclose(eps.grad.cpu().numpy()[lj], ref["vjp_eps"][lj], rtol=1e-10)
    pos = b.pos.clone().requires_grad_(True)
    f2 = H.nonbonded_forces_autograd(pos, b.charge, b.sigma, b.eps, b, p)
    with pytest.raises(NotImplementedError):
        f2.sum().backward()
