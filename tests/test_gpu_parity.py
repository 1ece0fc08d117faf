"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 path 1e-12 relative RMS force error; mixed path 1e-5 (single-
precision pair terms: per-pair relative error ~1e-7, see the erfc fit and the
fixed-point positions); binning and exclusion windows bit-exact.
"""

import dataclasses
import functools

import numpy as np
import pytest

import nbtest_util as U
from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

FP64_TOL = 1e-12
MIXED_TOL = 1e-5
KERNELS = [H.NB_KERNEL_ATOM, H.NB_KERNEL_CLUSTER, "cluster8", "cluster4_static", "half8", "half4_dynamic"]


def _assert_same(a, b, kernel, err_msg="", precision=H.NB_MIXED):
    """Bitwise equality, for every kernel and both precisions: the half-shell kernels add
    their atomic shares in 64-bit fixed point (two limbs on the FP64 path), whose sums do
    not depend on the order of the additions."""
    np.testing.assert_array_equal(a, b, err_msg=err_msg)


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def chain():
    return U.small_chain()


# --- binning: bit-exact ------------------------------------------------------------------

@pytest.mark.parametrize("divs", [(2, 2), (2, 8), (1, 1), (3, 3), (2, 3)])
@pytest.mark.parametrize("precision", [H.NB_MIXED, H.NB_FP64])
def test_binning_is_the_stable_counting_sort(divs, precision, chain):
    systems = [chain, U.cached_config(1), S.water_box(500, 25.0, seed=9)]
    _print_case("binning", divs=divs, precision=precision)
    out = U.gpu_eval(systems, precision, cell_div_xy=divs[0], cell_div_z=divs[1])
    ws = U.workspace_arrays(out)
    ref = U.oracle_binning(systems, precision, (divs[0], divs[0], divs[1]))
    np.testing.assert_array_equal(ws["cell_start"], ref["cell_start"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, 3], ref["order"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, :3], ref["sorted_fixed"])
    assert out["status"] == 0


@pytest.mark.parametrize("divs", [(2, 2), (2, 8), (2, 16), (3, 12), pytest.param((4, 16), marks=pytest.mark.skip(
    reason="took a GPU memory fault under a cross-lane (DPP) variant of the wave scans that has since "
           "been removed, without its cause shown; four cells per cutoff in x and y is now refused by "
           "the library (NB_ERR_ARG, checked on the CPU), so the case does not run (the multi-workgroup "
           "scan is covered by (2, 16) and (3, 12) here and by the million-atom tests)"))])
def test_binning_at_full_size_config2(divs):
    """(2, 2) and (2, 8) scan in the scatter launch (cell counts fit in LDS); (2, 16),
    17,914 cells, and (3, 12), 28,519 cells, take the multi-workgroup scan: two tiles of
    16,384 cells, the second partial."""
    s = U.cached_config(2)
    _print_case("binning-cfg2", divs=divs)
    out = U.gpu_eval(s, H.NB_MIXED, cell_div_xy=divs[0], cell_div_z=divs[1])
    ws = U.workspace_arrays(out)
    ref = U.oracle_binning([s], H.NB_MIXED, (divs[0], divs[0], divs[1]))
    np.testing.assert_array_equal(ws["cell_start"], ref["cell_start"])
    np.testing.assert_array_equal(ws["sorted_fixed"][:, 3], ref["order"])
    K = 8  # the mixed path's default cluster size
    nz = ws["dims"][2]
    cs = ref["cell_start"]
    col_atoms = cs[nz::nz] - cs[:-1:nz]
    expect = np.concatenate([[0], np.cumsum((col_atoms + K - 1) // K)])
    np.testing.assert_array_equal(ws["col_clu_start"], expect)


def test_exclusion_windows_are_exact(chain):
    from oracle import binning as OB
    systems = [chain, U.cached_config(1)]
    out = U.gpu_eval(systems, H.NB_FP64)
    ws = U.workspace_arrays(out)
    cat = S.concat_systems(systems)
    # the oracle takes global indices: shift each system's local partners
    idx = cat["excl_index"].copy()
    off = cat["excl_offset"]
    base = np.repeat(np.repeat([0, chain.n], [chain.n, U.cached_config(1).n]), np.diff(off))
    masks, far = OB.exclusion_windows(int(cat["atom_offset"][-1]), off, idx + base)
    np.testing.assert_array_equal(ws["excl_mask"], masks)
    assert not far.any()


def test_exclusion_windows_from_one_sided_lists(chain):
    """A pair listed in only one of its atoms' rows still excludes both ways: the
    windows equal the oracle's union and the two-sided list's, and so do the forces."""
    from oracle import binning as OB
    rng = np.random.default_rng(7)
    rows = [[] for _ in range(chain.n)]
    for i in range(chain.n):
        for k in range(chain.excl_offset[i], chain.excl_offset[i + 1]):
            j = int(chain.excl_index[k])
            if i < j or rng.random() < 0.5:  # always in the lower atom's row, half the time in both
                rows[i].append(j)
    off = np.zeros(chain.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    assert len(idx) < len(chain.excl_index)  # some pairs are now one-sided
    one = S.System(**{**chain.__dict__})
    one.excl_offset, one.excl_index = off, idx
    for precision in (H.NB_FP64, H.NB_MIXED):
        a = U.gpu_eval(chain, precision)
        b = U.gpu_eval(one, precision)
        masks, far = OB.exclusion_windows(one.n, off, idx)
        np.testing.assert_array_equal(U.workspace_arrays(b)["excl_mask"], masks)
        np.testing.assert_array_equal(U.workspace_arrays(b)["excl_mask"], U.workspace_arrays(a)["excl_mask"])
        np.testing.assert_array_equal(b["force"], a["force"])
        assert b["status"] == 0


@pytest.mark.parametrize("K", [4, 8])
def test_column_cluster_counts_are_exact(K, chain):
    # clusters are K consecutive sorted atoms of one (x, y) column: per column
    # ceil(count / K), scanned over the columns of every system in order
    systems = [chain, U.cached_config(1)]
    out = U.gpu_eval(systems, H.NB_MIXED, kernel=H.NB_KERNEL_CLUSTER, cluster_size=K)
    ws = U.workspace_arrays(out)
    ref = U.oracle_binning(systems, H.NB_MIXED, (2, 2, 8))
    from oracle import binning as OB
    per_col = []
    cell0 = 0
    for s in systems:
        dims = OB.grid_dims(s.box, s.cutoff, (2, 2, 8))
        nz = int(dims[2])
        for c in range(int(dims[0] * dims[1])):
            a0 = ref["cell_start"][cell0 + c * nz]
            a1 = ref["cell_start"][cell0 + (c + 1) * nz]
            per_col.append((a1 - a0 + K - 1) // K)
        cell0 += int(np.prod(dims))
    expect = np.concatenate([[0], np.cumsum(per_col)])
    np.testing.assert_array_equal(ws["col_clu_start"], expect)
    assert expect[-1] <= ws["n_clusters_max"]


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_split_and_cluster_size_give_the_same_forces(precision, K, chain):
    ref = U.oracle_for(chain, precision)
    tol = FP64_TOL if precision == H.NB_FP64 else MIXED_TOL
    outs = [U.gpu_eval(chain, precision, kernel=H.NB_KERNEL_CLUSTER, split=k, cluster_size=K, backward=True)
            for k in (1, 2, 3, 4, 8)]
    for o in outs:
        U.assert_forces(o["force"], ref["force"], precision, tol)
        assert U.rel_rms(o["grad_charge"], ref["phi"]) <= tol
        # mixed: on the scale of sum |E_i| (see test_forces_energy_virial_match_oracle)
        scale = abs(ref["energy_total"]) if precision == H.NB_FP64 else np.abs(ref["energy"]).sum()
        assert abs(o["energy"][0] - ref["energy_total"]) <= tol * scale
    for o in outs[1:]:  # splitting only reorders sums
        assert U.rel_rms(o["force"], outs[0]["force"]) <= (1e-13 if precision == H.NB_FP64 else 1e-6)


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_CLUSTER, H.NB_KERNEL_CLUSTER_HALF])
@pytest.mark.parametrize("split", [1, 3, 8])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_schedules_and_residency_give_bitwise_identical_results(precision, split, kernel, chain):
    """Every work item writes its own output slots, so neither the schedule (one item per
    wave, or persistent waves taking items from per-XCD counters) nor the number of
    resident workgroups may change a single bit; repeated dynamic runs neither.  On this
    input the static schedule of the mixed path runs the two-groups-per-pass kernel and
    the dynamic one the one-group kernel, so this also holds the two to the same bits.
    The half shell's atomic additions come in a different order on every run and
    schedule; its fixed-point sums may not change either."""
    runs = [U.gpu_eval(chain, precision, kernel=kernel, split=split, schedule=sch, wg_per_cu=w, backward=True)
            for sch, w in [(H.NB_SCHED_STATIC, 0), (H.NB_SCHED_DYNAMIC, 1), (H.NB_SCHED_DYNAMIC, 4),
                           (H.NB_SCHED_DYNAMIC, 16), (H.NB_SCHED_DYNAMIC, 32), (H.NB_SCHED_DYNAMIC, 4)]]
    for o in runs[1:]:
        for key in ("force", "energy", "virial", "grad_pos", "grad_charge", "grad_sigma", "grad_eps"):
            np.testing.assert_array_equal(o[key], runs[0][key], err_msg=key)
        assert o["status"] == 0


# --- forces, energies, virial --------------------------------------------------------------

@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("which", ["cfg1", "chain", "cfg2"])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_forces_energy_virial_match_oracle(which, precision, kernel, chain):
    s = {"cfg1": lambda: U.cached_config(1), "chain": lambda: chain, "cfg2": lambda: U.cached_config(2)}[which]()
    _print_case("forces", which=which, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True)
    ref = U.oracle_for(s, precision)
    tol = FP64_TOL if precision == H.NB_FP64 else MIXED_TOL
    print(f"  rel_rms={U.rel_rms(out['force'], ref['force']):.3e} "
          f"max_rel_atom={U.max_rel_atom(out['force'], ref['force']):.3e}")
    U.assert_forces(out["force"], ref["force"], precision, tol)
    if precision == H.NB_FP64:
        assert out["energy"][0] == pytest.approx(ref["energy_total"], rel=tol, abs=tol)
    else:
        # single-precision pair terms carry a relative error each, and the total is a small
        # difference of per-atom energies (water: about 100 times larger): compared on
        # the scale of sum |E_i|
        assert abs(out["energy"][0] - ref["energy_total"]) <= tol * np.abs(ref["energy"]).sum()
    assert U.rel_rms(out["virial"][0], ref["virial"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    # the energy call sums the same pairs in the same order; only the compiler's fusing of
    # multiply-adds may differ between the two kernels
    assert out["energy2"][0] == pytest.approx(out["energy"][0], rel=1e-12 if precision == H.NB_FP64 else 1e-7)
    assert out["status"] == 0


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_run_twice_is_bitwise_identical(precision, kernel, chain):
    a = U.gpu_eval(chain, precision, kernel=kernel)
    b = U.gpu_eval(chain, precision, kernel=kernel)
    _assert_same(a["force"], b["force"], kernel, precision=precision)
    # energy and virial come from per-item partials summed in a fixed order
    np.testing.assert_array_equal(a["energy"], b["energy"])
    np.testing.assert_array_equal(a["virial"], b["virial"])


@pytest.mark.parametrize("kernel", KERNELS)
def test_cell_grid_choice_does_not_change_the_result(kernel, chain):
    ref = U.oracle_for(chain, H.NB_FP64)
    ref32 = U.oracle_for(chain, H.NB_MIXED)
    for divs in [(1, 1), (2, 2), (2, 8), (3, 3), (3, 16), (1, 12)]:
        out = U.gpu_eval(chain, H.NB_FP64, cell_div_xy=divs[0], cell_div_z=divs[1], kernel=kernel)
        U.assert_forces(out["force"], ref["force"], H.NB_FP64, FP64_TOL)
        out = U.gpu_eval(chain, H.NB_MIXED, cell_div_xy=divs[0], cell_div_z=divs[1], kernel=kernel)
        U.assert_forces(out["force"], ref32["force"], H.NB_MIXED, MIXED_TOL)


def test_relabelled_atoms_give_permuted_forces(chain):
    rng = np.random.default_rng(3)
    p = rng.permutation(chain.n)
    inv = np.argsort(p)
    rows = [[] for _ in range(chain.n)]
    for i in range(chain.n):
        for k in range(chain.excl_offset[i], chain.excl_offset[i + 1]):
            rows[inv[i]].append(int(inv[chain.excl_index[k]]))
    off = np.zeros(chain.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in sorted(r)], np.int32)
    perm = S.System(**{**chain.__dict__})
    perm.pos, perm.charge, perm.type = chain.pos[p], chain.charge[p], chain.type[p]
    perm.excl_offset, perm.excl_index = off, idx
    a = U.gpu_eval(chain, H.NB_FP64)
    b = U.gpu_eval(perm, H.NB_FP64)
    np.testing.assert_allclose(b["force"], a["force"][p], rtol=0, atol=1e-12 * np.abs(a["force"]).max())
    c = U.gpu_eval(perm, H.NB_FP64, kernel=H.NB_KERNEL_ATOM)
    np.testing.assert_allclose(c["force"], a["force"][p], rtol=0, atol=1e-12 * np.abs(a["force"]).max())
    # relabelling moves some exclusions beyond the 64-atom window: the far path is exercised
    assert b["status"] == H.NB_STATUS_FAR_EXCLUSION


def _jittered_lattice(box, spacing, seed, cutoff, beta):
    """Atoms on a jittered lattice in an orthorhombic box (no close contacts), two LJ
    types, alternating charges, no exclusions."""
    rng = np.random.default_rng(seed)
    n = [int(L // spacing) for L in box]
    g = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
    pos = (g + 0.5) * (np.asarray(box) / n) + rng.uniform(-0.3, 0.3, g.shape)
    N = len(pos)
    return S.System(name="lattice", pos=np.mod(pos, box), charge=np.where(np.arange(N) % 2 == 0, 0.41, -0.41),
                    type=(rng.random(N) < 0.3).astype(np.int32), sigma=np.array([3.15, 2.5]),
                    eps=np.array([0.63, 0.2]), excl_offset=np.zeros(N + 1, np.int32),
                    excl_index=np.zeros(0, np.int32), box=np.asarray(box, np.float64), cutoff=cutoff,
                    beta=beta, seed=seed)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("cutoff,beta", [(9.0, 0.0), (7.0, 0.34), (12.0, 0.25), (9.0, 0.5)])
def test_non_cubic_box_other_cutoffs_and_bare_coulomb(cutoff, beta, precision, kernel):
    """A 30 x 36 x 42 A box (a different fixed-point scale per axis and a different cell
    grid per axis), cutoffs of 7 and 12 A, beta = 0 (the truncated bare Coulomb term,
    erfc = 1), and beta R = 4.5 (beyond the short FP64 erfc table)."""
    s = _jittered_lattice((30.0, 36.0, 42.0), 2.5, seed=21, cutoff=cutoff, beta=beta)
    _print_case("non_cubic", cutoff=cutoff, beta=beta, precision=precision, kernel=kernel, n=s.n)
    out = U.gpu_eval(s, precision, kernel=kernel, energy_call=True)
    ref = U.oracle_for(s, precision)
    tol = FP64_TOL if precision == H.NB_FP64 else MIXED_TOL
    err = U.rel_rms(out["force"], ref["force"])
    # With beta = 0 the total is a small remainder of pair terms thousands of times
    # larger, so the energy is judged on the scale of the per-atom energies.
    scale = float(np.abs(ref["energy"]).sum())
    e_err = abs(out["energy"][0] - ref["energy_total"]) / scale
    v_err = U.rel_rms(out["virial"][0], ref["virial"])
    print(f"  rel_rms={err:.3e} energy/sum|E_i|={e_err:.3e} virial={v_err:.3e}")
    U.assert_forces(out["force"], ref["force"], precision, tol)
    assert e_err <= tol
    assert v_err <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert U.rel_rms(out["atom_energy"], ref["energy"]) <= (1e-11 if precision == H.NB_FP64 else 1e-5)
    assert out["status"] == 0


@pytest.mark.parametrize("kernel", [H.NB_KERNEL_CLUSTER, "cluster4_static", "half8", H.NB_KERNEL_ATOM])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_net_force_vanishes_and_translation_leaves_the_result(precision, kernel, chain):
    """Newton's third law (the forces sum to zero up to rounding) and invariance under a
    translation that is not a box multiple (every fixed-point coordinate changes)."""
    out = U.gpu_eval(chain, precision, kernel=kernel)
    f = out["force"].reshape(-1, 3)
    f_rms = float(np.sqrt(np.mean(np.sum(f * f, axis=1))))
    net = float(np.linalg.norm(f.sum(axis=0))) / (chain.n * f_rms)
    print(f"  net force / (N F_rms) = {net:.3e}")
    assert net <= (1e-14 if precision == H.NB_FP64 else 1e-7)
    moved = S.System(**{**chain.__dict__})
    moved.pos = np.mod(chain.pos + np.array([1.2345, -5.6789, 9.1011]), chain.box)
    out2 = U.gpu_eval(moved, precision, kernel=kernel)
    # the mixed path sees the FP32 rounding of the moved positions: compare with the oracle
    ref = U.oracle_for(moved, precision)
    tol = FP64_TOL if precision == H.NB_FP64 else MIXED_TOL
    U.assert_forces(out2["force"], ref["force"], precision, tol)
    assert U.rel_rms(out2["force"], out["force"]) <= (1e-12 if precision == H.NB_FP64 else 1e-5)
    assert out2["energy"][0] == pytest.approx(out["energy"][0], rel=1e-12 if precision == H.NB_FP64 else 1e-5)


# --- batches -------------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_batch_equals_each_system_alone(precision, kernel, chain):
    systems = [S.water_box(300, 20.0, seed=1), chain, S.water_box(1200, 26.0, seed=2),
               S.solvated_chain(30.0, 80, 800, seed=4, cutoff=9.0, beta=0.34)]
    out = U.gpu_eval(systems, precision, kernel=kernel)
    off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
    for k, s in enumerate(systems):
        alone = U.gpu_eval(s, precision, kernel=kernel)
        _assert_same(out["force"][off[k]:off[k + 1]], alone["force"], kernel, precision=precision)
        assert out["energy"][k] == alone["energy"][0]
        np.testing.assert_array_equal(out["virial"][k], alone["virial"][0])


# --- edge cases ----------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", KERNELS)
def test_tiny_and_empty_systems(kernel):
    two = S.System(name="two", pos=np.array([[1.0, 1.0, 1.0], [4.0, 1.0, 1.5]]), charge=np.array([0.5, -0.5]),
                   type=np.array([0, 0], np.int32), sigma=np.array([3.0]), eps=np.array([0.4]),
                   excl_offset=np.zeros(3, np.int32), excl_index=np.zeros(0, np.int32),
                   box=np.array([20.0, 21.0, 22.0]), cutoff=9.0, beta=0.3, seed=0)
    empty = S.System(name="empty", pos=np.zeros((0, 3)), charge=np.zeros(0), type=np.zeros(0, np.int32),
                     sigma=np.array([3.0]), eps=np.array([0.4]), excl_offset=np.zeros(1, np.int32),
                     excl_index=np.zeros(0, np.int32), box=np.array([20.0, 20.0, 20.0]), cutoff=9.0,
                     beta=0.3, seed=0)
    out = U.gpu_eval([two, empty, two], H.NB_FP64, kernel=kernel)
    ref = U.oracle_for(two, H.NB_FP64)
    np.testing.assert_allclose(out["force"][:2], ref["force"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out["force"][2:], ref["force"], rtol=1e-13, atol=1e-13)
    assert out["energy"][1] == 0.0 and not out["virial"][1].any()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_positions_outside_the_box_are_wrapped(precision, kernel, chain):
    moved = S.System(**{**chain.__dict__})
    shift = np.zeros_like(chain.pos)
    shift[::2] = chain.box * np.array([2, -3, 1])
    shift[1::5] = -chain.box * np.array([1, 1, 4])
    moved.pos = chain.pos + shift
    out = U.gpu_eval(moved, precision, kernel=kernel)
    ref = U.oracle_for(moved, precision)
    U.assert_forces(out["force"], ref["force"], precision, 1e-11 if precision == H.NB_FP64 else MIXED_TOL)


def test_device_status_bits():
    s = S.water_box(200, 19.0, seed=5)
    bad = S.System(**{**s.__dict__})
    bad.pos = s.pos.copy()
    bad.pos[7, 1] = np.nan
    bad.type = s.type.copy()
    bad.type[3] = 17
    out = U.gpu_eval(bad, H.NB_FP64)
    assert out["status"] & H.NB_STATUS_NONFINITE_POS
    assert out["status"] & H.NB_STATUS_BAD_TYPE
    bad2 = S.System(**{**s.__dict__})
    bad2.excl_index = s.excl_index.copy()
    bad2.excl_index[5] = 10 ** 6
    out = U.gpu_eval(bad2, H.NB_FP64)
    assert out["status"] & H.NB_STATUS_BAD_EXCLUSION


# --- adjoint -------------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
@pytest.mark.parametrize("which", ["chain", "cfg3"])
def test_backward_matches_oracle_gradients(precision, which, kernel, chain):
    s = chain if which == "chain" else U.cached_config(3)
    _print_case("backward", which=which, precision=precision, kernel=kernel)
    g = 1.7
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True, grad_energy=[g])
    ref = U.oracle_for(s, precision)
    tol = 1e-11 if precision == H.NB_FP64 else MIXED_TOL
    U.assert_forces(out["grad_pos"], -g * ref["force"], precision, tol)
    assert U.rel_rms(out["grad_charge"], g * ref["phi"]) <= tol
    present = np.unique(s.type)
    lj = present[s.eps[present] > 0]
    np.testing.assert_allclose(out["grad_sigma"][lj], g * ref["dsigma"][lj], rtol=tol * 10, atol=tol)
    np.testing.assert_allclose(out["grad_eps"][lj], g * ref["deps"][lj], rtol=tol * 10, atol=tol)
    assert np.all(out["grad_eps"][s.eps == 0] == 0.0)


def test_autograd_function_and_fd_of_the_fp64_energy(chain):
    b = H.device_batch([chain], dtype=torch.float64)
    p = H.make_params(chain.cutoff, chain.beta, H.NB_FP64)
    pos = b.pos.clone().requires_grad_(True)
    q = b.charge.clone().requires_grad_(True)
    sig = b.sigma.clone().requires_grad_(True)
    eps = b.eps.clone().requires_grad_(True)
    E = H.nonbonded_energy_autograd(pos, q, sig, eps, b, p)
    E.sum().backward()
    h = 1e-4

    def energy(**kw):
        args = dict(pos=b.pos, q=b.charge, sig=b.sigma, eps=b.eps)
        args.update(kw)
        with torch.no_grad():
            return float(H.nonbonded_energy_autograd(args["pos"], args["q"], args["sig"], args["eps"], b, p)[0])

    rng = np.random.default_rng(0)
    n_ok = 0
    for i in rng.choice(chain.n, 25, replace=False):
        d = chain.pos - chain.pos[i]
        d -= chain.box * np.rint(d / chain.box)
        r = np.sqrt((d * d).sum(1))
        if np.any(np.abs(r - chain.cutoff) <= 2 * h):
            continue  # a probe would cross the hard cutoff
        for a in range(3):
            pp = b.pos.clone(); pp[i, a] += h
            pm = b.pos.clone(); pm[i, a] -= h
            fd = (energy(pos=pp) - energy(pos=pm)) / (2 * h)
            assert fd == pytest.approx(float(pos.grad[i, a]), rel=1e-4, abs=1e-4)
        n_ok += 1
    assert n_ok >= 10
    for t in np.unique(chain.type):
        if chain.eps[t] <= 0:
            continue
        sp = b.sigma.clone(); sp[t] += h
        sm = b.sigma.clone(); sm[t] -= h
        assert (energy(sig=sp) - energy(sig=sm)) / (2 * h) == pytest.approx(float(sig.grad[t]), rel=1e-4, abs=1e-5)
        ep = b.eps.clone(); ep[t] += h
        em = b.eps.clone(); em[t] -= h
        assert (energy(eps=ep) - energy(eps=em)) / (2 * h) == pytest.approx(float(eps.grad[t]), rel=1e-4, abs=1e-5)
    for i in (0, 40, 300):
        qp = b.charge.clone(); qp[i] += h
        qm = b.charge.clone(); qm[i] -= h
        assert (energy(q=qp) - energy(q=qm)) / (2 * h) == pytest.approx(float(q.grad[i]), rel=1e-5, abs=1e-6)


# --- full-size configurations --------------------------------------------------------------

def test_config5_mixed_against_sampled_oracle_and_fp64_gpu():
    s = U.cached_config(5)
    _print_case("cfg5", n=s.n)
    mixed = U.gpu_eval(s, H.NB_MIXED)
    mixed_atom = U.gpu_eval(s, H.NB_MIXED, kernel=H.NB_KERNEL_ATOM)
    assert U.rel_rms(mixed_atom["force"], mixed["force"]) <= 1e-6
    # Kernel error only: the FP64 path on the same FP32-rounded coordinates and charges
    # (FP32 rounding of the inputs at L = 215 A is itself ~1e-5 relative in the forces).
    fp64_same_in = U.gpu_eval(s.rounded(np.float32), H.NB_FP64)
    err = U.rel_rms(mixed["force"], fp64_same_in["force"])
    print(f"  mixed vs fp64 gpu rel_rms={err:.3e} "
          f"max_rel_atom={U.max_rel_atom(mixed['force'], fp64_same_in['force']):.3e}")
    assert err <= MIXED_TOL
    rows = np.random.default_rng(5).choice(s.n, 96, replace=False)
    ref32 = U.oracle_for(s, H.NB_MIXED, rows=rows)
    U.assert_forces(mixed["force"][rows], ref32["force"], H.NB_MIXED, MIXED_TOL)
    U.assert_forces(fp64_same_in["force"][rows], ref32["force"], H.NB_FP64, FP64_TOL)
    fp64 = U.gpu_eval(s, H.NB_FP64)
    ref64 = U.oracle_for(s, H.NB_FP64, rows=rows)
    U.assert_forces(fp64["force"][rows], ref64["force"], H.NB_FP64, FP64_TOL)


@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_config5_adjoint_identities_sampled_oracle_and_fp64_gpu(precision):
    """The adjoint at full size (999,999 atoms, R = 12 A), where the oracle can only take
    sampled rows.  Besides dE/dq on sampled rows and dE/dx = -F, three identities pin the
    per-type and per-charge sums at any size.  E_LJ is homogeneous of degree one in the
    eps_t (eps_ij = sqrt(eps_ti eps_tj)), so sum_t eps_t dE/deps_t = E_LJ; scaling every
    sigma_t scales every sigma_ij, and s dE_LJ/ds = sum over pairs of (12 A - 6 B) = the
    trace of the LJ virial; E_C is quadratic in the charges, so sum_i q_i dE/dq_i = 2 E_C.
    E_C and the Coulomb virial come from the same call with every eps_t set to zero."""
    s = U.cached_config(5).rounded(np.float32)  # one set of inputs for both paths
    _print_case("cfg5-adjoint", n=s.n, precision=precision)
    out = U.gpu_eval(s, precision, backward=True)
    s_c = dataclasses.replace(s, eps=np.zeros_like(s.eps))
    coul = U.gpu_eval(s_c, precision)
    e, e_c = float(out["energy"][0]), float(coul["energy"][0])
    tr_w = float(np.trace(out["virial"].reshape(3, 3)))
    tr_wc = float(np.trace(coul["virial"].reshape(3, 3)))
    q_sum = float(np.dot(s.charge, out["grad_charge"]))
    eps_sum = float(np.dot(s.eps, out["grad_eps"]))
    sig_sum = float(np.dot(s.sigma, out["grad_sigma"]))
    print(f"  q.dE/dq={q_sum:.10e} 2E_C={2 * e_c:.10e}  eps.dE/deps={eps_sum:.10e} E_LJ={e - e_c:.10e}  "
          f"sig.dE/dsig={sig_sum:.10e} trW_LJ={tr_w - tr_wc:.10e}")
    if precision == H.NB_FP64:
        assert q_sum == pytest.approx(2 * e_c, rel=1e-10)
        assert eps_sum == pytest.approx(e - e_c, rel=1e-10)
        assert sig_sum == pytest.approx(tr_w - tr_wc, rel=1e-10)
    else:
        # E_C and E_LJ are small differences of per-atom sums 100-1000 times larger, so
        # per-pair errors of ~1e-7 are compared on the scale of those sums: sum |q_i phi_i|
        # for the charges, and the per-type tolerance of the other adjoint tests (1e-4)
        # for eps and sigma.
        scale = float(np.abs(s.charge * out["grad_charge"]).sum())
        print(f"  sum|q phi|={scale:.4e}")
        assert abs(q_sum - 2 * e_c) <= MIXED_TOL * scale
        assert eps_sum == pytest.approx(e - e_c, rel=10 * MIXED_TOL)
        assert sig_sum == pytest.approx(tr_w - tr_wc, rel=10 * MIXED_TOL)
    assert U.rel_rms(out["grad_pos"], -out["force"]) <= (1e-12 if precision == H.NB_FP64 else 1e-6)
    rows = np.random.default_rng(55).choice(s.n, 96, replace=False)
    ref = O.evaluate_system(s, rows=rows, ke=H.COULOMB_K)
    assert U.rel_rms(out["grad_charge"][rows], ref["phi"]) <= (FP64_TOL if precision == H.NB_FP64 else MIXED_TOL)
    U.assert_forces(out["grad_pos"][rows], -ref["force"], precision, FP64_TOL if precision == H.NB_FP64 else MIXED_TOL)
    if precision == H.NB_MIXED:  # against the FP64 GPU path on the same inputs
        ref64 = U.gpu_eval(s, H.NB_FP64, backward=True)
        for k in ("grad_pos", "grad_charge"):
            err = U.rel_rms(out[k], ref64[k])
            print(f"  {k}: mixed vs fp64 gpu rel_rms={err:.3e}")
            assert err <= MIXED_TOL
        lj = s.eps > 0
        np.testing.assert_allclose(out["grad_sigma"][lj], ref64["grad_sigma"][lj], rtol=10 * MIXED_TOL)
        np.testing.assert_allclose(out["grad_eps"][lj], ref64["grad_eps"][lj], rtol=10 * MIXED_TOL)


def test_pair_kernels_refuse_a_workspace_built_for_another_kernel(chain):
    b = H.device_batch([chain], dtype=torch.float32)
    p_atom = H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, kernel=H.NB_KERNEL_ATOM)
    p_clu = H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, kernel=H.NB_KERNEL_CLUSTER)
    ws = torch.zeros(max(H.workspace_bytes(b, p_atom), H.workspace_bytes(b, p_clu)), dtype=torch.uint8,
                     device="cuda")
    force = torch.full((chain.n, 3), 7.0, dtype=torch.float64, device="cuda")
    energy = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    # never built: nothing is written and the status says so
    H.nonbonded_forces(b, p_clu, ws, force, energy)
    assert H.read_status(ws) & H.NB_STATUS_NOT_BUILT
    assert float(force.abs().min()) == 7.0 and float(energy[0]) == 7.0
    H.build_cells(b, p_atom, ws)
    H.nonbonded_forces(b, p_clu, ws, force, energy)
    assert H.read_status(ws) & H.NB_STATUS_NOT_BUILT
    H.build_cells(b, p_clu, ws)
    H.nonbonded_forces(b, p_clu, ws, force, energy)
    assert H.read_status(ws) == 0


def test_pair_kernels_refuse_a_build_for_another_cluster_size_or_split(chain):
    """The build writes each launch slot's work item for one cluster size and one number of
    items per cluster; a forces call with another of either must not run on it."""
    b = H.device_batch([chain], dtype=torch.float32)
    p8 = H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, cluster_size=8, split=1)
    others = [H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, cluster_size=8, split=2),
              H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, cluster_size=4, split=1)]
    ws = torch.zeros(max(H.workspace_bytes(b, p) for p in [p8] + others), dtype=torch.uint8, device="cuda")
    force = torch.full((chain.n, 3), 7.0, dtype=torch.float64, device="cuda")
    energy = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    for p in others:
        H.build_cells(b, p8, ws)
        H.nonbonded_forces(b, p, ws, force, energy)
        assert H.read_status(ws) & H.NB_STATUS_NOT_BUILT
        assert float(force.abs().min()) == 7.0 and float(force.abs().max()) == 7.0 and float(energy[0]) == 7.0
    for p in [p8] + others:
        H.build_cells(b, p, ws)
        H.nonbonded_forces(b, p, ws, force, energy)
        assert H.read_status(ws) == 0
        assert U.rel_rms(force.cpu().numpy(), U.oracle_for(chain, H.NB_MIXED)["force"]) <= MIXED_TOL


def test_half_shell_kernel_refuses_a_build_without_its_accumulators(chain):
    """A build for the full-shell kernel does not zero the half-shell accumulators, so
    the half-shell kernel must neither run on it nor write the outputs."""
    b = H.device_batch([chain], dtype=torch.float32)
    p_clu = H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, kernel=H.NB_KERNEL_CLUSTER)
    p_half = H.make_params(chain.cutoff, chain.beta, H.NB_MIXED, kernel=H.NB_KERNEL_CLUSTER_HALF)
    assert H.workspace_bytes(b, p_half) > H.workspace_bytes(b, p_clu)
    ws = torch.full((H.workspace_bytes(b, p_half),), 0x7F, dtype=torch.uint8, device="cuda")  # not zero
    force = torch.full((chain.n, 3), 7.0, dtype=torch.float64, device="cuda")
    energy = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    H.build_cells(b, p_clu, ws)
    H.nonbonded_forces(b, p_half, ws, force, energy)
    assert H.read_status(ws) & H.NB_STATUS_NOT_BUILT
    assert float(force.abs().min()) == 7.0 and float(force.abs().max()) == 7.0 and float(energy[0]) == 7.0
    H.build_cells(b, p_half, ws)
    H.nonbonded_forces(b, p_half, ws, force, energy)
    assert H.read_status(ws) == 0
    ref = U.oracle_for(chain, H.NB_MIXED)
    assert U.rel_rms(force.cpu().numpy(), ref["force"]) <= MIXED_TOL
    # the accumulators were zeroed again: a second call gives the same forces
    f1 = force.clone()
    H.nonbonded_forces(b, p_half, ws, force, energy)
    _assert_same(force.cpu().numpy(), f1.cpu().numpy(), "half8")


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_half_shell_agrees_with_full_shell(precision, K):
    """Each pair once, the other atom's share added by atomics, against each pair twice:
    the same pair terms summed in another grouping, over splits and both schedules."""
    s = U.cached_config(2)
    full = U.gpu_eval(s, precision, kernel=H.NB_KERNEL_CLUSTER, cluster_size=K, energy_call=True)
    tol = 1e-13 if precision == H.NB_FP64 else 3e-6
    for split, sch in [(1, H.NB_SCHED_STATIC), (2, H.NB_SCHED_STATIC), (3, H.NB_SCHED_DYNAMIC),
                       (8, H.NB_SCHED_DYNAMIC)]:
        _print_case("half_vs_full", precision=precision, K=K, split=split, schedule=sch, n=s.n)
        half = U.gpu_eval(s, precision, kernel=H.NB_KERNEL_CLUSTER_HALF, cluster_size=K, split=split,
                          schedule=sch, energy_call=True)
        err = U.rel_rms(half["force"], full["force"])
        print(f"  half vs full rel_rms={err:.3e}")
        assert err <= tol
        assert half["energy"][0] == pytest.approx(full["energy"][0], rel=tol)
        assert half["energy2"][0] == pytest.approx(full["energy2"][0], rel=tol)
        assert U.rel_rms(half["virial"][0], full["virial"][0]) <= tol
        assert U.rel_rms(half["atom_energy"], full["atom_energy"]) <= tol
        assert half["status"] == 0


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [H.NB_FP64, H.NB_MIXED])
def test_many_types_use_the_global_type_table(precision, kernel, chain):
    # 20 types: more than the cluster kernel keeps in LDS
    rng = np.random.default_rng(8)
    s = S.System(**{**chain.__dict__})
    s.sigma = np.concatenate([chain.sigma, rng.uniform(2.5, 3.8, 10)])
    s.eps = np.concatenate([chain.eps, rng.uniform(0.1, 0.9, 10)])
    s.type = chain.type.copy()
    s.type[:chain.n_solute] = rng.integers(2, 20, chain.n_solute)
    out = U.gpu_eval(s, precision, kernel=kernel, backward=True)
    ref = U.oracle_for(s, precision)
    tol = FP64_TOL if precision == H.NB_FP64 else MIXED_TOL
    assert U.rel_rms(out["force"], ref["force"]) <= tol
    lj = np.unique(s.type)
    lj = lj[s.eps[lj] > 0]
    np.testing.assert_allclose(out["grad_sigma"][lj], ref["dsigma"][lj], rtol=max(tol * 10, 1e-10), atol=tol)


# --- the batched form: 64 uneven replicas in one launch ---------------------------------------

@functools.lru_cache(maxsize=None)
def _replicas():
    return S.config4()


def test_batch64_against_sampled_oracle_and_fp64_gpu():
    """807,400 atoms in 64 boxes of 3k-30k atoms, one build and one forces call: forces
    of 16 sampled atoms per replica against the FP64 oracle, every atom's mixed force
    against the FP64 GPU path on the same rounded inputs, per-replica energies."""
    systems = list(_replicas())
    _print_case("batch64", n=sum(s.n for s in systems))
    mixed = U.gpu_eval(systems, H.NB_MIXED)
    rounded = [s.rounded(np.float32) for s in systems]
    fp64 = U.gpu_eval(rounded, H.NB_FP64, energy_call=True)
    assert mixed["status"] == 0 and fp64["status"] == 0
    err = U.rel_rms(mixed["force"], fp64["force"])
    print(f"  mixed vs fp64 gpu rel_rms={err:.3e}")
    assert err <= MIXED_TOL
    # A replica's real-space energy is a sum of per-atom energies of both signs that
    # nearly cancel (totals of a few hundred kJ/mol against sums of |E_i| near 1e5), so
    # the single-precision pair terms' error is bounded on the scale of the summands.
    off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
    scale = np.array([np.abs(fp64["atom_energy"][off[k]:off[k + 1]]).sum() for k in range(len(systems))])
    dev = np.abs(mixed["energy"] - fp64["energy"]) / scale
    print(f"  energy |mixed - fp64| / sum|E_i| max={dev.max():.3e}")
    assert dev.max() <= MIXED_TOL
    rng = np.random.default_rng(4)
    off = 0
    num = den = 0.0
    for s in rounded:
        rows = np.sort(rng.choice(s.n, 16, replace=False))
        ref = O.evaluate_system(s, rows=rows, ke=H.COULOMB_K)
        assert U.rel_rms(fp64["force"][off + rows], ref["force"]) <= FP64_TOL
        num += float(np.sum((mixed["force"][off + rows] - ref["force"]) ** 2))
        den += float(np.sum(ref["force"] ** 2))
        off += s.n
    assert np.sqrt(num / den) <= MIXED_TOL


@pytest.mark.parametrize("sched", [H.NB_SCHED_STATIC, H.NB_SCHED_DYNAMIC])
def test_batch64_subset_equals_each_replica_alone(sched):
    systems = list(_replicas())
    order = np.argsort([s.n for s in systems])
    pick = [systems[k] for k in (order[0], order[20], order[45], order[-1])]
    out = U.gpu_eval(pick, H.NB_MIXED, schedule=sched, split=2)
    off = np.concatenate([[0], np.cumsum([s.n for s in pick])])
    for k, s in enumerate(pick):
        alone = U.gpu_eval(s, H.NB_MIXED, schedule=sched, split=2)
        np.testing.assert_array_equal(out["force"][off[k]:off[k + 1]], alone["force"])
        assert out["energy"][k] == alone["energy"][0]


def test_autotuner_choice_is_correct_and_cached(chain, tmp_path, monkeypatch):
    from paper_0902_0827_amd import autotune as A
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "tune.json"))
    b = H.device_batch([chain], dtype=torch.float32)
    p, rec = A.tune(b, chain.cutoff, chain.beta, H.NB_MIXED, reps=3, warmup=1, budget_s=20.0)
    assert len(rec["tried"]) >= 5 and not rec.get("cached")
    force, energy, vir, ws = H.evaluate(b, p)
    ref = U.oracle_for(chain, H.NB_MIXED)
    assert U.rel_rms(force.cpu().numpy(), ref["force"]) <= MIXED_TOL
    assert H.read_status(ws) == 0
    p2, rec2 = A.tune(b, chain.cutoff, chain.beta, H.NB_MIXED)
    assert rec2.get("cached") and all(getattr(p2, k) == getattr(p, k) for k in A.PARAM_KEYS)
