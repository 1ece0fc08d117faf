"""Host-side checks of the C ABI (no GPU): the library loads, exports every symbol that
include/nbhip.h declares, sizes workspaces, and rejects bad arguments before it
enqueues any work."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_0902_0827_amd import nbhip as H
from paper_0902_0827_amd import systems as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbhip.h")

pytestmark = pytest.mark.skipif(not os.path.exists(H.LIB_PATH), reason="libnbhip.so not built")

FAKE = 0x7F0000000000  # any non-null value: host validation never dereferences device pointers


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:nb_status|const char \*)\s*(nb_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = H.load_library()
    names = declared_functions()
    assert set(names) == set(H.EXPORTED)
    for n in names:
        assert hasattr(lib, n)


def fake_system(n_atoms=(648,), L=18.6, n_types=2):
    offs = np.concatenate([[0], np.cumsum(n_atoms)]).astype(np.int64)
    box = np.tile(np.asarray(L, float).reshape(-1, 3) if np.ndim(L) else np.array([[L, L, L]]),
                  (len(n_atoms), 1)) if np.ndim(L) < 2 else np.asarray(L, float)
    s = H.nb_system()
    s.n_systems = len(n_atoms)
    s._off = np.ascontiguousarray(offs)
    s._box = np.ascontiguousarray(box.reshape(-1))
    s.atom_offset = s._off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    s.box = s._box.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s.pos = s.charge = s.type = s.lj_sigma = s.lj_eps = s.excl_offset = s.excl_index = FAKE
    s.pos_is_f64 = 0
    s.n_types = n_types
    return s


def ws_bytes(sys, prm):
    lib = H.load_library()
    n = ctypes.c_size_t()
    code = lib.nb_workspace_bytes(ctypes.byref(sys), ctypes.byref(prm), ctypes.byref(n))
    return code, n.value


def test_workspace_bytes_scales_with_the_system():
    prm = H.make_params(9.0, 0.34)
    code, small = ws_bytes(fake_system((648,)), prm)
    assert code == H.NB_OK and small > 0
    code, big = ws_bytes(fake_system((23600,), L=60.0), prm)
    assert code == H.NB_OK and big > 20 * small
    code, batch = ws_bytes(fake_system((3000, 5000, 0, 7000), L=40.0), prm)
    assert code == H.NB_OK


def test_half_shell_kernel_adds_one_accumulator_per_atom():
    """The half-shell kernel's workspace holds 32 more bytes per atom (force and energy
    accumulators), rounded up to the 256-byte alignment of every array."""
    s = fake_system((23600,), L=60.0)
    code, full = ws_bytes(s, H.make_params(9.0, 0.34, kernel=H.NB_KERNEL_CLUSTER))
    assert code == H.NB_OK
    code, half = ws_bytes(s, H.make_params(9.0, 0.34, kernel=H.NB_KERNEL_CLUSTER_HALF))
    assert code == H.NB_OK
    assert half - full == (32 * 23600 + 255) // 256 * 256


def test_fp64_half_shell_holds_two_limbs_per_component():
    """The FP64 path's half-shell accumulators are 64-bit fixed point in two limbs: 64 bytes
    per atom instead of the mixed path's 32."""
    s = fake_system((23600,), L=60.0)
    code, full = ws_bytes(s, H.make_params(9.0, 0.34, H.NB_FP64, kernel=H.NB_KERNEL_CLUSTER, cluster_size=8))
    assert code == H.NB_OK
    code, half = ws_bytes(s, H.make_params(9.0, 0.34, H.NB_FP64, kernel=H.NB_KERNEL_CLUSTER_HALF, cluster_size=8))
    assert code == H.NB_OK
    assert half - full == (64 * 23600 + 255) // 256 * 256


def test_layout_reports_the_grid():
    lib = H.load_library()
    lay = H.nb_layout()
    prm = H.make_params(9.0, 0.34, cell_div_z=8)
    assert lib.nb_workspace_layout(ctypes.byref(fake_system((23600,), L=60.0)), ctypes.byref(prm),
                                   ctypes.byref(lay)) == H.NB_OK
    assert list(lay.dims) == [13, 13, 53]
    assert lay.n_cells == 13 * 13 * 53 and lay.n_atoms == 23600
    for off in (lay.off_cell_start, lay.off_sorted_fixed, lay.off_sorted_pos64, lay.off_excl_mask):
        assert off % 256 == 0


@pytest.mark.parametrize("mutate,code", [
    (lambda s, p: setattr(p, "cutoff", 9.3), H.NB_ERR_BOX),          # R = L/2
    (lambda s, p: setattr(p, "cutoff", -1.0), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "ewald_beta", -0.1), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "precision", 7), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "cell_div_xy", 9), H.NB_ERR_ARG),
    # four cells per cutoff in x and y is refused: the pair kernel's run table is sized
    # for (2k+1)^2 <= 49 neighbour columns
    (lambda s, p: setattr(p, "cell_div_xy", 4), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "kernel", 99), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "kernel", H.NB_KERNEL_CLUSTER_HALF + 1), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "split", 9), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "cluster_size", 6), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "schedule", 3), H.NB_ERR_ARG),
    (lambda s, p: setattr(p, "wg_per_cu", 33), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "n_types", 0), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "n_types", H.NB_MAX_TYPES + 1), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "n_systems", 0), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "pos", None), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "excl_index", None), H.NB_ERR_ARG),
    (lambda s, p: setattr(s, "pos_is_f64", 3), H.NB_ERR_ARG),
    (lambda s, p: s._box.__setitem__(1, -5.0), H.NB_ERR_BOX),
    (lambda s, p: s._box.__setitem__(2, float("nan")), H.NB_ERR_BOX),
    (lambda s, p: s._off.__setitem__(1, -3), H.NB_ERR_ARG),
])
def test_host_validation_rejects(mutate, code):
    s = fake_system((648,))
    p = H.make_params(9.0, 0.34)
    mutate(s, p)
    got, _ = ws_bytes(s, p)
    assert got == code
    assert H.last_error() != ""


def test_workspace_checks_happen_before_any_launch():
    lib = H.load_library()
    s = fake_system((648,))
    p = H.make_params(9.0, 0.34)
    code, need = ws_bytes(s, p)
    assert code == H.NB_OK
    # too small, NULL, misaligned: all refused on the host (no device is touched)
    assert lib.nb_build_cells(ctypes.byref(s), ctypes.byref(p), FAKE, need - 1, None) == H.NB_ERR_WORKSPACE
    assert lib.nb_build_cells(ctypes.byref(s), ctypes.byref(p), None, need, None) == H.NB_ERR_WORKSPACE
    assert lib.nb_build_cells(ctypes.byref(s), ctypes.byref(p), FAKE + 8, need, None) == H.NB_ERR_WORKSPACE
    assert "too small" in H.last_error() or "aligned" in H.last_error()
    assert lib.nb_nonbonded_forces(ctypes.byref(s), ctypes.byref(p), FAKE, need, None, None, None, None) \
        == H.NB_ERR_ARG  # force is required
    assert lib.nb_nonbonded_backward(ctypes.byref(s), ctypes.byref(p), FAKE, need, None, None, None, None,
                                     None, None) == H.NB_ERR_ARG  # grad_energy is required
    assert lib.nb_nonbonded_energy(ctypes.byref(s), ctypes.byref(p), FAKE, need, None, None, None) == H.NB_ERR_ARG
    assert lib.nb_ewald_corrections(ctypes.byref(s), ctypes.byref(p), FAKE, need, None, None, None, None) \
        == H.NB_ERR_ARG  # force is required
    assert lib.nb_ewald_corrections(ctypes.byref(s), ctypes.byref(p), FAKE, need - 1, FAKE, None, None, None) \
        == H.NB_ERR_WORKSPACE


def test_workload_generators_have_the_documented_shapes():
    s1 = S.config1()
    assert s1.n == 648 and np.allclose(s1.box, 18.6)
    oh = np.linalg.norm(s1.pos[1] - s1.pos[0])
    hh = np.linalg.norm(s1.pos[2] - s1.pos[1])
    assert oh == pytest.approx(0.9572, abs=1e-9) and hh == pytest.approx(1.5139, abs=1e-4)
    assert abs(s1.charge.sum()) < 1e-12
    s2 = S.config2()
    assert s2.n == 23600 and s2.n_solute == 2000
    assert s2.n / np.prod(s2.box) == pytest.approx(0.10926, rel=1e-3)
    assert abs(s2.charge.sum()) < 1e-9
    # every exclusion within the 64-atom index window
    rows = np.repeat(np.arange(s2.n), np.diff(s2.excl_offset))
    assert np.abs(s2.excl_index - rows).max() <= 2


def test_pair_timer_argument_checks():
    lib = H.load_library()
    assert lib.nb_pair_timer_start(0) == H.NB_ERR_ARG
    assert lib.nb_pair_timer_start(65537) == H.NB_ERR_ARG
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.nb_pair_timer_stop(ctypes.byref(ms), ctypes.byref(n)) == H.NB_ERR_ARG  # never started
    assert "not started" in H.last_error()


def test_pme_workspace_and_argument_checks():
    """Grid and argument checks come before any HIP or FFT-library call.  The work area
    of the FFT plans is part of the workspace; its size needs the plans, so a valid grid
    asks the current device (NB_ERR_HIP here, without one)."""
    lib = H.load_library()
    s = fake_system((648, 100))
    p = H.make_params(9.0, 0.34)
    G = ctypes.c_int32 * 3
    n = ctypes.c_size_t()
    P = lambda g: ctypes.cast(g, ctypes.POINTER(ctypes.c_int32))
    for bad in [(3, 32, 32), (32, 0, 32), (32, 32, 1025)]:
        assert lib.nb_pme_workspace_bytes(ctypes.byref(s), P(G(*bad)), ctypes.byref(n)) == H.NB_ERR_ARG
        assert "grid" in H.last_error()
    code = lib.nb_pme_workspace_bytes(ctypes.byref(s), P(G(32, 30, 27)), ctypes.byref(n))
    # two systems, each a real grid, its half spectrum and its convolution partials (10
    # per 256 elements), then the FFT work area
    spec = 32 * 30 * (27 // 2 + 1)
    up = lambda x: (x + 255) // 256 * 256
    grids = up(2 * 8 * 32 * 30 * 27) + up(2 * 16 * spec) + up(2 * 8 * 10 * ((spec + 255) // 256))
    if code == H.NB_OK:
        assert n.value >= grids
    else:
        assert code == H.NB_ERR_HIP and "nb_pme_workspace_bytes" in H.last_error()
    g = P(G(32, 30, 27))
    # workspaces smaller than the grids alone are refused before the plans are made
    assert lib.nb_pme_reciprocal(ctypes.byref(s), ctypes.byref(p), g, FAKE, grids - 1, FAKE, None, None, None) \
        == H.NB_ERR_WORKSPACE
    assert lib.nb_pme_reciprocal(ctypes.byref(s), ctypes.byref(p), g, FAKE + 8, grids, FAKE, None, None, None) \
        == H.NB_ERR_WORKSPACE
    assert lib.nb_pme_reciprocal(ctypes.byref(s), ctypes.byref(p), g, FAKE, grids, None, None, None, None) \
        == H.NB_ERR_ARG  # force is required
    assert lib.nb_pme_reciprocal(ctypes.byref(s), ctypes.byref(p), P(G(2, 30, 27)), FAKE, grids, FAKE, None, None,
                                 None) == H.NB_ERR_ARG
    p0 = H.make_params(9.0, 0.0)
    assert lib.nb_pme_reciprocal(ctypes.byref(s), ctypes.byref(p0), g, FAKE, grids, FAKE, None, None, None) \
        == H.NB_ERR_ARG and "beta" in H.last_error()


_CATCH_ALL_CHILD = r"""
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_0902_0827_amd import nbhip as H
lib = H.load_library()
B = 4_000_000  # the plan's per-system table (128 bytes each) needs 512 MB of host memory
off = np.zeros(B + 1, np.int64)
box = np.full(3 * B, 2.5)
s = H.nb_system()
s.n_systems = B
s.atom_offset = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
s.box = box.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
s.lj_sigma = s.lj_eps = 0x7F0000000000
s.n_types = 2
p = H.make_params(1.0, 0.34, cell_div_xy=1, cell_div_z=1)  # 8 cells per system
n = ctypes.c_size_t()
ok = lib.nb_workspace_bytes(ctypes.byref(s), ctypes.byref(p), ctypes.byref(n))
# cap the address space just above what the process maps now: the next large host
# allocation inside the library fails with std::bad_alloc
with open("/proc/self/statm") as f:
    pages = int(f.read().split()[0])
cap = pages * resource.getpagesize() + (64 << 20)
resource.setrlimit(resource.RLIMIT_AS, (cap, cap))
code = lib.nb_workspace_bytes(ctypes.byref(s), ctypes.byref(p), ctypes.byref(n))
print(ok, code, H.last_error())
"""


def test_no_exception_crosses_the_abi():
    """An allocation failure inside an entry point comes back as NB_ERR_HOST with a
    message, not as a C++ exception through the C interface (which would abort)."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, "-c", _CATCH_ALL_CHILD, ROOT], capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    ok, code, msg = res.stdout.strip().split(" ", 2)
    assert int(ok) == H.NB_OK  # the same call succeeds without the cap
    assert int(code) == H.NB_ERR_HOST and "out of host memory" in msg


def test_noalloc_entry_point_refuses_batches_beyond_its_scratch():
    """The allocation-free entry point checks the batch's workspace against its fixed
    scratch size before any HIP call."""
    lib = H.load_library()
    s = fake_system((300_000, 300_000), L=150.0)
    p = H.make_params(9.0, 0.34)
    code = lib.nb_nonbonded_forces_noalloc(ctypes.byref(s), ctypes.byref(p), FAKE, None, None, None)
    assert code == H.NB_ERR_CAPACITY and "allocation-free" in H.last_error()
    assert lib.nb_nonbonded_forces_noalloc(ctypes.byref(s), ctypes.byref(p), None, None, None, None) \
        == H.NB_ERR_ARG  # force is required


def test_force_field_options_are_validated_on_the_host():
    lib = H.load_library()
    n = ctypes.c_size_t()
    s = fake_system((648,))
    ok = lambda p: lib.nb_workspace_bytes(ctypes.byref(s), ctypes.byref(p), ctypes.byref(n))
    assert ok(H.make_params(9.0, 0.34, lj_switch_on=7.5)) == H.NB_OK
    assert ok(H.make_params(9.0, 0.34, lj_switch_on=9.0)) == H.NB_ERR_ARG  # r_on must be below R
    assert ok(H.make_params(9.0, 0.34, lj_switch_on=-1.0)) == H.NB_ERR_ARG
    assert ok(H.make_params(9.0, 0.34, scale14_lj=float("nan"))) == H.NB_ERR_ARG
    # the per-atom kernel supports neither option
    assert ok(H.make_params(9.0, 0.34, kernel=H.NB_KERNEL_ATOM, lj_switch_on=7.5)) == H.NB_ERR_ARG
    assert "per-atom" in H.last_error()
    base = ws_bytes(s, H.make_params(9.0, 0.34))[1]
    s.pair14_offset = FAKE
    assert ok(H.make_params(9.0, 0.34)) == H.NB_ERR_ARG  # offsets without indices
    s.pair14_index = FAKE
    assert ok(H.make_params(9.0, 0.34)) == H.NB_OK
    assert n.value >= base + 16 * 648  # one 128-bit 1-4 window per atom
    assert ok(H.make_params(9.0, 0.34, kernel=H.NB_KERNEL_ATOM)) == H.NB_ERR_ARG


def test_force_vjp_host_checks():
    """The force VJP needs v and a cluster kernel; both are checked before any launch."""
    lib = H.load_library()
    s = fake_system((648,))
    p = H.make_params(9.0, 0.34)
    code, need = ws_bytes(s, p)
    assert code == H.NB_OK
    assert lib.nb_nonbonded_force_vjp(ctypes.byref(s), ctypes.byref(p), FAKE, need, None, None, None, None,
                                      None) == H.NB_ERR_ARG  # v is required
    assert lib.nb_nonbonded_force_vjp(ctypes.byref(s), ctypes.byref(p), FAKE, need - 1, FAKE, None, None, None,
                                      None) == H.NB_ERR_WORKSPACE
    pa = H.make_params(9.0, 0.34, kernel=H.NB_KERNEL_ATOM)
    code, need_a = ws_bytes(s, pa)
    assert code == H.NB_OK
    assert lib.nb_nonbonded_force_vjp(ctypes.byref(s), ctypes.byref(pa), FAKE, need_a, FAKE, None, None, None,
                                      None) == H.NB_ERR_ARG
    assert "cluster kernel" in H.last_error()


def _md_topo(n_waters=216):
    t = H.nb_md_topology()
    t.mass = FAKE
    t.n_waters = n_waters
    t.water_o = FAKE
    t.water_r_oh, t.water_r_hh = 0.9572, 1.5139
    t.n_bonds = t.n_angles = 0
    return t


def test_md_calls_validate_on_the_host():
    """MD workspace size and argument checks (no GPU: no PME grid, fake device pointers)."""
    lib = H.load_library()
    s = fake_system((648,))
    p = H.make_params(9.0, 0.34)
    md = H.make_md_params(0.004, 300.0, 1.0, 7)
    n = ctypes.c_size_t()
    call = lambda: lib.nb_md_workspace_bytes(ctypes.byref(s), ctypes.byref(p), ctypes.byref(md), ctypes.byref(n))
    assert call() == H.NB_ERR_ARG and "pos_is_f64" in H.last_error()  # the MD state is FP64
    s.pos_is_f64 = 1
    assert call() == H.NB_OK
    nb = ws_bytes(s, p)[1]
    assert n.value >= nb + 2 * 3 * 8 * 648 + 648  # short-range and bonded forces, roles
    need = n.value
    md.dt = 0.0
    assert call() == H.NB_ERR_ARG
    md.dt = 0.004
    md.gamma = -1.0
    assert call() == H.NB_ERR_ARG
    md.gamma = 1.0
    md.pme_grid[0] = 2  # a grid below 4 points
    md.pme_grid[1] = md.pme_grid[2] = 32
    assert call() == H.NB_ERR_ARG
    md.pme_grid[0] = md.pme_grid[1] = md.pme_grid[2] = 0
    topo = _md_topo()
    run = lambda t, ws, size, pos, vel, n_steps: lib.nb_md_run(
        ctypes.byref(s), ctypes.byref(p), t, ctypes.byref(md), ws, size, pos, vel, 0, n_steps, None, None)
    assert run(None, FAKE, need, FAKE, FAKE, 1) == H.NB_ERR_ARG                    # no topology
    assert run(ctypes.byref(topo), FAKE, need - 1, FAKE, FAKE, 1) == H.NB_ERR_WORKSPACE
    assert run(ctypes.byref(topo), FAKE, need, FAKE + 8, FAKE, 1) == H.NB_ERR_ARG  # pos is not sys->pos
    assert run(ctypes.byref(topo), FAKE, need, FAKE, None, 1) == H.NB_ERR_ARG      # no velocities
    assert run(ctypes.byref(topo), FAKE, need, FAKE, FAKE, -1) == H.NB_ERR_ARG
    bad = _md_topo()
    bad.water_r_hh = 2.0  # not a triangle with r_oh = 0.9572
    assert run(ctypes.byref(bad), FAKE, need, FAKE, FAKE, 1) == H.NB_ERR_ARG
    bad = _md_topo(217)   # more waters than 648 atoms hold
    assert run(ctypes.byref(bad), FAKE, need, FAKE, FAKE, 1) == H.NB_ERR_ARG
    bad = _md_topo()
    bad.n_bonds = 3       # bonds without arrays
    assert run(ctypes.byref(bad), FAKE, need, FAKE, FAKE, 1) == H.NB_ERR_ARG
    assert lib.nb_md_forces(ctypes.byref(s), ctypes.byref(p), ctypes.byref(topo), ctypes.byref(md), FAKE, need,
                            None, None, None) == H.NB_ERR_ARG  # force is required


def test_md_topology_generator():
    s = S.config2()
    t = S.md_topology(s)
    assert t["water_o"].size == (s.n - s.n_solute) // 3 == 7200
    assert len(t["bonds"]) == s.n_solute - 1 and len(t["angles"]) == s.n_solute - 2
    # the generator's waters hold the rigid geometry the constraints keep
    o = t["water_o"]
    d = lambda a, b: np.linalg.norm(S._minimage(s.pos[a] - s.pos[b], s.box), axis=1)
    assert np.allclose(d(o, o + 1), t["r_oh"], atol=1e-12) and np.allclose(d(o + 1, o + 2), t["r_hh"], atol=1e-12)
    cat = S.concat_topologies([t, t], [s.n, s.n])
    assert cat["water_o"][7200] == s.n + o[0] and cat["bonds"][len(t["bonds"])][0] == s.n
