"""Python binding of libnbhip.so (include/nbhip.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module turns torch
tensors into the C structs and raw device pointers the C ABI takes, and enqueues
on torch's current HIP stream.  There is no fallback: if the library is not
built, or no GPU is present, the calls raise.

Names follow the C ABI: ``workspace_bytes``, ``build_cells``, ``nonbonded_forces``,
``nonbonded_energy``, ``nonbonded_backward``, ``read_status``, ``last_error``.
``NonbondedEnergy`` wraps forward energy + hand-written adjoint as a
``torch.autograd.Function``.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NBHIP_LIB selects another build of the library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("NBHIP_LIB") or os.path.join(_HERE, "libnbhip.so")

# Coulomb constant k_e = e^2 N_A / (4 pi eps0), CODATA 2018, kJ mol^-1 A e^-2.
COULOMB_K = 1389.35457644382

NB_OK, NB_ERR_ARG, NB_ERR_BOX, NB_ERR_WORKSPACE, NB_ERR_HIP, NB_ERR_CAPACITY, NB_ERR_HOST = range(7)
NB_FP64, NB_MIXED = 0, 1
NB_SCHED_AUTO, NB_SCHED_STATIC, NB_SCHED_DYNAMIC = 0, 1, 2
NB_KERNEL_AUTO, NB_KERNEL_ATOM, NB_KERNEL_CLUSTER, NB_KERNEL_CLUSTER_HALF = 0, 1, 2, 3
NB_STATUS_NONFINITE_POS = 0x1
NB_STATUS_BAD_TYPE = 0x2
NB_STATUS_BAD_EXCLUSION = 0x4
NB_STATUS_FAR_EXCLUSION = 0x8
NB_STATUS_NOT_BUILT = 0x10
NB_STATUS_FAR_PAIR14 = 0x20
NB_STATUS_BAD_TOPOLOGY = 0x40
NB_MAX_TYPES = 64

EXPORTED = ("nb_workspace_bytes", "nb_build_cells", "nb_nonbonded_forces", "nb_nonbonded_energy",
            "nb_nonbonded_backward", "nb_read_status", "nb_last_error", "nb_workspace_layout",
            "nb_pair_timer_start", "nb_pair_timer_stop", "nb_ewald_corrections",
            "nb_pme_workspace_bytes", "nb_pme_reciprocal", "nb_nonbonded_forces_noalloc",
            "nb_nonbonded_force_vjp", "nb_md_workspace_bytes", "nb_md_forces", "nb_md_run")


class NbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nbhip error {code}: {msg}")
        self.code = code


class nb_system(ctypes.Structure):
    _fields_ = [
        ("n_systems", ctypes.c_int32),
        ("atom_offset", ctypes.POINTER(ctypes.c_int64)),
        ("box", ctypes.POINTER(ctypes.c_double)),
        ("pos", ctypes.c_void_p),
        ("pos_is_f64", ctypes.c_int32),
        ("charge", ctypes.c_void_p),
        ("type", ctypes.c_void_p),
        ("lj_sigma", ctypes.c_void_p),
        ("lj_eps", ctypes.c_void_p),
        ("n_types", ctypes.c_int32),
        ("excl_offset", ctypes.c_void_p),
        ("excl_index", ctypes.c_void_p),
        ("pair14_offset", ctypes.c_void_p),
        ("pair14_index", ctypes.c_void_p),
    ]


class nb_params(ctypes.Structure):
    _fields_ = [
        ("cutoff", ctypes.c_double),
        ("ewald_beta", ctypes.c_double),
        ("coulomb_k", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("cell_div_xy", ctypes.c_int32),
        ("cell_div_z", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("split", ctypes.c_int32),
        ("cluster_size", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("wg_per_cu", ctypes.c_int32),
        ("lj_switch_on", ctypes.c_double),
        ("scale14_lj", ctypes.c_double),
        ("scale14_coul", ctypes.c_double),
        ("table", ctypes.c_int32),
        ("table_size", ctypes.c_int32),
    ]


class nb_md_topology(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_void_p),
        ("n_waters", ctypes.c_int64),
        ("water_o", ctypes.c_void_p),
        ("water_r_oh", ctypes.c_double),
        ("water_r_hh", ctypes.c_double),
        ("n_bonds", ctypes.c_int64),
        ("bond_atoms", ctypes.c_void_p),
        ("bond_k", ctypes.c_void_p),
        ("bond_r0", ctypes.c_void_p),
        ("n_angles", ctypes.c_int64),
        ("angle_atoms", ctypes.c_void_p),
        ("angle_k", ctypes.c_void_p),
        ("angle_theta0", ctypes.c_void_p),
    ]


class nb_md_params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("temperature", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("pme_grid", ctypes.c_int32 * 3),
        ("reserved", ctypes.c_int32),
        ("aux_stream", ctypes.c_void_p),
    ]


class nb_layout(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int64),
        ("n_cells", ctypes.c_int64),
        ("dims", ctypes.c_int32 * 3),
        ("off_cell_start", ctypes.c_int64),
        ("off_sorted_fixed", ctypes.c_int64),
        ("off_sorted_pos64", ctypes.c_int64),
        ("off_excl_mask", ctypes.c_int64),
        ("off_status", ctypes.c_int64),
        ("n_columns", ctypes.c_int64),
        ("n_clusters_max", ctypes.c_int64),
        ("off_col_clu_start", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnbhip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0902_0827_amd.build_lib`")
    lib = ctypes.CDLL(path)
    S, P, V = ctypes.POINTER(nb_system), ctypes.POINTER(nb_params), ctypes.c_void_p
    sz = ctypes.c_size_t
    lib.nb_workspace_bytes.argtypes = [S, P, ctypes.POINTER(sz)]
    lib.nb_build_cells.argtypes = [S, P, V, sz, V]
    lib.nb_nonbonded_forces.argtypes = [S, P, V, sz, V, V, V, V]
    lib.nb_nonbonded_energy.argtypes = [S, P, V, sz, V, V, V]
    lib.nb_nonbonded_backward.argtypes = [S, P, V, sz, V, V, V, V, V, V]
    lib.nb_nonbonded_force_vjp.argtypes = [S, P, V, sz, V, V, V, V, V]
    MT, MP = ctypes.POINTER(nb_md_topology), ctypes.POINTER(nb_md_params)
    lib.nb_md_workspace_bytes.argtypes = [S, P, MP, ctypes.POINTER(sz)]
    lib.nb_md_forces.argtypes = [S, P, MT, MP, V, sz, V, V, V]
    lib.nb_md_run.argtypes = [S, P, MT, MP, V, sz, V, V, ctypes.c_int64, ctypes.c_int64, V, V]
    lib.nb_ewald_corrections.argtypes = [S, P, V, sz, V, V, V, V]
    lib.nb_nonbonded_forces_noalloc.argtypes = [S, P, V, V, V, V]
    G = ctypes.POINTER(ctypes.c_int32)
    lib.nb_pme_workspace_bytes.argtypes = [S, G, ctypes.POINTER(ctypes.c_size_t)]
    lib.nb_pme_reciprocal.argtypes = [S, P, G, V, sz, V, V, V, V]
    lib.nb_read_status.argtypes = [V, V, ctypes.POINTER(ctypes.c_uint32)]
    lib.nb_workspace_layout.argtypes = [S, P, ctypes.POINTER(nb_layout)]
    lib.nb_pair_timer_start.argtypes = [ctypes.c_int32]
    lib.nb_pair_timer_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTED:
        getattr(lib, name).restype = ctypes.c_int if name != "nb_last_error" else ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().nb_last_error().decode()


def _check(code: int):
    if code != NB_OK:
        raise NbError(code, last_error())


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def make_params(cutoff: float, beta: float, precision: int = NB_MIXED, coulomb_k: float = COULOMB_K,
                cell_div_xy: int = 0, cell_div_z: int = 0, kernel: int = NB_KERNEL_AUTO, split: int = 0,
                cluster_size: int = 0, schedule: int = 0, wg_per_cu: int = 0, lj_switch_on: float = 0.0,
                scale14_lj: float = 1.0, scale14_coul: float = 1.0, table: int = 0,
                table_size: int = 0) -> nb_params:
    return nb_params(float(cutoff), float(beta), float(coulomb_k), int(precision), int(cell_div_xy),
                     int(cell_div_z), int(kernel), int(split), int(cluster_size), int(schedule), int(wg_per_cu),
                     float(lj_switch_on), float(scale14_lj), float(scale14_coul), int(table), int(table_size))


@dataclass
class DeviceBatch:
    """Torch device tensors (and host arrays) of a batch of systems, plus its nb_system."""

    pos: "object"          # [N,3] float32 or float64 cuda tensor
    charge: "object"       # [N] same dtype as pos
    type: "object"         # [N] int32
    sigma: "object"        # [T] float64
    eps: "object"          # [T] float64
    excl_offset: "object"  # [N+1] int32
    excl_index: "object"   # [n_excl] int32 (at least one element)
    atom_offset: np.ndarray
    box: np.ndarray        # [B,3] float64
    pair14_offset: "object" = None  # [N+1] int32, or None
    pair14_index: "object" = None   # [n_14] int32 (at least one element), or None
    _struct: nb_system = field(default=None, repr=False)

    @property
    def n_systems(self) -> int:
        return int(self.atom_offset.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_offset[-1])

    def struct(self) -> nb_system:
        """The nb_system view; refreshed on each call so that tensor replacements are seen."""
        self._off_c = np.ascontiguousarray(self.atom_offset, np.int64)
        self._box_c = np.ascontiguousarray(self.box, np.float64).reshape(-1)
        s = nb_system()
        s.n_systems = self.n_systems
        s.atom_offset = self._off_c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        s.box = self._box_c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        import torch
        s.pos = _ptr(self.pos)
        s.pos_is_f64 = 1 if self.pos.dtype == torch.float64 else 0
        s.charge = _ptr(self.charge)
        s.type = _ptr(self.type)
        s.lj_sigma = _ptr(self.sigma)
        s.lj_eps = _ptr(self.eps)
        s.n_types = int(self.sigma.shape[0])
        s.excl_offset = _ptr(self.excl_offset)
        s.excl_index = _ptr(self.excl_index)
        s.pair14_offset = _ptr(self.pair14_offset)
        s.pair14_index = _ptr(self.pair14_index)
        self._struct = s
        return s


def device_batch(systems: Sequence, dtype=None, device: str = "cuda") -> DeviceBatch:
    """Upload one or more ``systems.System`` objects (packed back to back)."""
    import torch
    from . import systems as S
    systems = list(systems) if isinstance(systems, (list, tuple)) else [systems]
    cat = S.concat_systems(systems)
    dt = torch.float32 if dtype is None else dtype
    ei = cat["excl_index"] if cat["excl_index"].size else np.zeros(1, np.int32)
    return DeviceBatch(
        pos=torch.tensor(cat["pos"], dtype=dt, device=device),
        charge=torch.tensor(cat["charge"], dtype=dt, device=device),
        type=torch.tensor(cat["type"], dtype=torch.int32, device=device),
        sigma=torch.tensor(cat["sigma"], dtype=torch.float64, device=device),
        eps=torch.tensor(cat["eps"], dtype=torch.float64, device=device),
        excl_offset=torch.tensor(cat["excl_offset"], dtype=torch.int32, device=device),
        excl_index=torch.tensor(ei, dtype=torch.int32, device=device),
        atom_offset=cat["atom_offset"].astype(np.int64),
        box=cat["box"].astype(np.float64),
        pair14_offset=None if cat["pair14_offset"] is None else
        torch.tensor(cat["pair14_offset"], dtype=torch.int32, device=device),
        pair14_index=None if cat["pair14_offset"] is None else
        torch.tensor(cat["pair14_index"] if cat["pair14_index"].size else np.zeros(1, np.int32),
                     dtype=torch.int32, device=device),
    )


# --- the C ABI, one function each ------------------------------------------------------------

def workspace_bytes(batch: DeviceBatch, params: nb_params) -> int:
    lib = load_library()
    n = ctypes.c_size_t()
    _check(lib.nb_workspace_bytes(ctypes.byref(batch.struct()), ctypes.byref(params), ctypes.byref(n)))
    return int(n.value)


def alloc_workspace(batch: DeviceBatch, params: nb_params):
    """A uint8 cuda tensor of the required size (torch allocations are 256-byte aligned)."""
    import torch
    ws = torch.empty(max(workspace_bytes(batch, params), 1), dtype=torch.uint8, device=batch.pos.device)
    assert ws.data_ptr() % 256 == 0
    return ws


def workspace_layout(batch: DeviceBatch, params: nb_params) -> nb_layout:
    lib = load_library()
    lay = nb_layout()
    _check(lib.nb_workspace_layout(ctypes.byref(batch.struct()), ctypes.byref(params), ctypes.byref(lay)))
    return lay


def build_cells(batch: DeviceBatch, params: nb_params, ws, stream=None):
    lib = load_library()
    _check(lib.nb_build_cells(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                              _stream(stream)))


def nonbonded_forces(batch: DeviceBatch, params: nb_params, ws, force, energy=None, virial=None, stream=None):
    lib = load_library()
    _check(lib.nb_nonbonded_forces(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                                   _ptr(force), _ptr(energy), _ptr(virial), _stream(stream)))


def nonbonded_forces_noalloc(batch: DeviceBatch, params: nb_params, force, energy=None, virial=None, stream=None):
    """Build + forces on the library's own scratch array (nb_nonbonded_forces_noalloc)."""
    lib = load_library()
    _check(lib.nb_nonbonded_forces_noalloc(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(force),
                                           _ptr(energy), _ptr(virial), _stream(stream)))


def ewald_corrections(batch: DeviceBatch, params: nb_params, ws, force, energy=None, virial=None, stream=None):
    """Excluded-pair and self corrections of the Ewald sum (nb_ewald_corrections)."""
    lib = load_library()
    _check(lib.nb_ewald_corrections(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                                    _ptr(force), _ptr(energy), _ptr(virial), _stream(stream)))


def _grid(grid):
    g = (ctypes.c_int32 * 3)(*[int(k) for k in grid])
    return ctypes.cast(g, ctypes.POINTER(ctypes.c_int32)), g


def pme_workspace_bytes(batch: DeviceBatch, grid) -> int:
    lib = load_library()
    n = ctypes.c_size_t()
    gp, _keep = _grid(grid)
    _check(lib.nb_pme_workspace_bytes(ctypes.byref(batch.struct()), gp, ctypes.byref(n)))
    return int(n.value)


def alloc_pme_workspace(batch: DeviceBatch, grid):
    """A uint8 cuda tensor for nb_pme_reciprocal on this batch and grid."""
    import torch
    ws = torch.empty(max(pme_workspace_bytes(batch, grid), 1), dtype=torch.uint8, device=batch.pos.device)
    assert ws.data_ptr() % 256 == 0
    return ws


def pme_reciprocal(batch: DeviceBatch, params: nb_params, grid, ws, force, energy=None, virial=None, stream=None):
    """Reciprocal part of the Ewald sum by smooth PME on a K1 x K2 x K3 grid (nb_pme_reciprocal)."""
    lib = load_library()
    gp, _keep = _grid(grid)
    _check(lib.nb_pme_reciprocal(ctypes.byref(batch.struct()), ctypes.byref(params), gp, _ptr(ws), ws.numel(),
                                 _ptr(force), _ptr(energy), _ptr(virial), _stream(stream)))


def nonbonded_energy(batch: DeviceBatch, params: nb_params, ws, energy, atom_energy=None, stream=None):
    lib = load_library()
    _check(lib.nb_nonbonded_energy(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                                   _ptr(energy), _ptr(atom_energy), _stream(stream)))


def nonbonded_backward(batch: DeviceBatch, params: nb_params, ws, grad_energy, grad_pos=None,
                       grad_charge=None, grad_sigma=None, grad_eps=None, stream=None):
    lib = load_library()
    _check(lib.nb_nonbonded_backward(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                                     _ptr(grad_energy), _ptr(grad_pos), _ptr(grad_charge), _ptr(grad_sigma),
                                     _ptr(grad_eps), _stream(stream)))


def nonbonded_force_vjp(batch: DeviceBatch, params: nb_params, ws, v, grad_charge=None, grad_sigma=None,
                        grad_eps=None, stream=None):
    """dL/dq [N], dL/dsigma [T], dL/deps [T] of L = sum_i v_i . F_i (any output may be None)."""
    lib = load_library()
    _check(lib.nb_nonbonded_force_vjp(ctypes.byref(batch.struct()), ctypes.byref(params), _ptr(ws), ws.numel(),
                                      _ptr(v), _ptr(grad_charge), _ptr(grad_sigma), _ptr(grad_eps),
                                      _stream(stream)))


# --- molecular dynamics --------------------------------------------------------------------

@dataclass
class DeviceTopology:
    """Device tensors of an MD topology (systems.md_topology / concat_topologies layout)."""

    mass: "object"
    water_o: "object"
    r_oh: float
    r_hh: float
    bonds: "object"
    bond_k: "object"
    bond_r0: "object"
    angles: "object"
    angle_k: "object"
    angle_theta0: "object"

    def struct(self) -> nb_md_topology:
        t = nb_md_topology()
        t.mass = _ptr(self.mass)
        t.n_waters = int(self.water_o.numel())
        t.water_o = _ptr(self.water_o) if t.n_waters else None
        t.water_r_oh, t.water_r_hh = float(self.r_oh), float(self.r_hh)
        t.n_bonds = int(self.bonds.shape[0])
        t.bond_atoms = _ptr(self.bonds) if t.n_bonds else None
        t.bond_k = _ptr(self.bond_k) if t.n_bonds else None
        t.bond_r0 = _ptr(self.bond_r0) if t.n_bonds else None
        t.n_angles = int(self.angles.shape[0])
        t.angle_atoms = _ptr(self.angles) if t.n_angles else None
        t.angle_k = _ptr(self.angle_k) if t.n_angles else None
        t.angle_theta0 = _ptr(self.angle_theta0) if t.n_angles else None
        return t


def device_topology(topo: dict, device: str = "cuda") -> DeviceTopology:
    import torch
    f64 = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float64, device=device)
    i32 = lambda a: torch.tensor(np.asarray(a, np.int32), dtype=torch.int32, device=device)
    return DeviceTopology(mass=f64(topo["mass"]), water_o=i32(topo["water_o"]), r_oh=topo["r_oh"],
                          r_hh=topo["r_hh"], bonds=i32(topo["bonds"]).reshape(-1, 2), bond_k=f64(topo["bond_k"]),
                          bond_r0=f64(topo["bond_r0"]), angles=i32(topo["angles"]).reshape(-1, 3),
                          angle_k=f64(topo["angle_k"]), angle_theta0=f64(topo["angle_theta0"]))


def make_md_params(dt: float, temperature: float = 300.0, gamma: float = 1.0, seed: int = 1,
                   pme_grid=(0, 0, 0), aux_stream=None) -> nb_md_params:
    """aux_stream: None, or a torch.cuda.Stream for the reciprocal part (run concurrently)."""
    m = nb_md_params()
    m.dt, m.temperature, m.gamma, m.seed = float(dt), float(temperature), float(gamma), int(seed)
    for a in range(3):
        m.pme_grid[a] = int(pme_grid[a])
    m.reserved = 0
    m.aux_stream = None if aux_stream is None else int(aux_stream.cuda_stream)
    m._aux = aux_stream  # keeps the stream alive as long as the params
    return m


def md_workspace_bytes(batch: DeviceBatch, params: nb_params, md: nb_md_params) -> int:
    n = ctypes.c_size_t()
    _check(load_library().nb_md_workspace_bytes(ctypes.byref(batch.struct()), ctypes.byref(params),
                                                ctypes.byref(md), ctypes.byref(n)))
    return int(n.value)


def alloc_md_workspace(batch: DeviceBatch, params: nb_params, md: nb_md_params):
    import torch
    ws = torch.empty(max(md_workspace_bytes(batch, params, md), 1), dtype=torch.uint8, device=batch.pos.device)
    assert ws.data_ptr() % 256 == 0
    return ws


def md_forces(batch: DeviceBatch, params: nb_params, topo: DeviceTopology, md: nb_md_params, ws, force,
              energy=None, stream=None):
    _check(load_library().nb_md_forces(ctypes.byref(batch.struct()), ctypes.byref(params),
                                       ctypes.byref(topo.struct()), ctypes.byref(md), _ptr(ws), ws.numel(),
                                       _ptr(force), _ptr(energy), _stream(stream)))


def md_run(batch: DeviceBatch, params: nb_params, topo: DeviceTopology, md: nb_md_params, ws, vel,
           first_step: int, n_steps: int, energy=None, stream=None):
    """n_steps integrator steps in place on batch.pos (float64) and vel."""
    _check(load_library().nb_md_run(ctypes.byref(batch.struct()), ctypes.byref(params),
                                    ctypes.byref(topo.struct()), ctypes.byref(md), _ptr(ws), ws.numel(),
                                    _ptr(batch.pos), _ptr(vel), int(first_step), int(n_steps), _ptr(energy),
                                    _stream(stream)))


def read_status(ws, stream=None) -> int:
    lib = load_library()
    flags = ctypes.c_uint32()
    _check(lib.nb_read_status(_ptr(ws), _stream(stream), ctypes.byref(flags)))
    return int(flags.value)


def pair_timer_start(capacity: int = 4096):
    """Record HIP events around every following pair-kernel launch (up to `capacity`)."""
    _check(load_library().nb_pair_timer_start(int(capacity)))


def pair_timer_stop():
    """Stop recording; returns (summed pair-kernel milliseconds, recorded launches)."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load_library().nb_pair_timer_stop(ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


# --- convenience --------------------------------------------------------------------------

def evaluate(batch: DeviceBatch, params: nb_params, ws=None, virial: bool = True):
    """build_cells + nonbonded_forces; returns (force [N,3], energy [B], virial [B,3,3] or None, ws)."""
    import torch
    if ws is None:
        ws = alloc_workspace(batch, params)
    dev = batch.pos.device
    B = batch.n_systems
    force = torch.empty((batch.n_atoms, 3), dtype=torch.float64, device=dev)
    energy = torch.empty(B, dtype=torch.float64, device=dev)
    vir = torch.empty((B, 3, 3), dtype=torch.float64, device=dev) if virial else None
    build_cells(batch, params, ws)
    nonbonded_forces(batch, params, ws, force, energy, vir)
    return force, energy, vir, ws


def _rebatch(batch: DeviceBatch, pos, charge, sigma, eps) -> DeviceBatch:
    import torch
    return DeviceBatch(pos=pos.detach().contiguous(), charge=charge.detach().contiguous(), type=batch.type,
                       sigma=sigma.detach().to(torch.float64).contiguous(),
                       eps=eps.detach().to(torch.float64).contiguous(),
                       excl_offset=batch.excl_offset, excl_index=batch.excl_index,
                       atom_offset=batch.atom_offset, box=batch.box,
                       pair14_offset=batch.pair14_offset, pair14_index=batch.pair14_index)


def _autograd():
    import torch

    class NonbondedEnergy(torch.autograd.Function):
        """E_b(pos, charge, sigma, eps) for every system b of ``batch``, with the hand-written adjoint.

        ``pos``/``charge`` must be the tensors held by ``batch`` (or the same shape and dtype:
        they replace them for this call).  Returns a float64 tensor [B].
        """

        @staticmethod
        def forward(ctx, pos, charge, sigma, eps, batch: DeviceBatch, params: nb_params):
            b = _rebatch(batch, pos, charge, sigma, eps)
            ws = alloc_workspace(b, params)
            build_cells(b, params, ws)
            energy = torch.empty(b.n_systems, dtype=torch.float64, device=pos.device)
            nonbonded_energy(b, params, ws, energy)
            ctx.batch, ctx.params, ctx.ws = b, params, ws
            ctx.dtypes = (pos.dtype, charge.dtype, sigma.dtype, eps.dtype)
            return energy

        @staticmethod
        def backward(ctx, grad_energy):
            b, params, ws = ctx.batch, ctx.params, ctx.ws
            dev = b.pos.device
            g = grad_energy.detach().to(torch.float64).contiguous()
            need = ctx.needs_input_grad
            gp = torch.empty((b.n_atoms, 3), dtype=torch.float64, device=dev) if need[0] else None
            gq = torch.empty(b.n_atoms, dtype=torch.float64, device=dev) if need[1] else None
            gs = torch.empty(b.sigma.shape[0], dtype=torch.float64, device=dev) if need[2] else None
            ge = torch.empty(b.sigma.shape[0], dtype=torch.float64, device=dev) if need[3] else None
            nonbonded_backward(b, params, ws, g, gp, gq, gs, ge)
            pd, qd, sd, ed = ctx.dtypes
            return (None if gp is None else gp.to(pd), None if gq is None else gq.to(qd),
                    None if gs is None else gs.to(sd), None if ge is None else ge.to(ed), None, None)

    class NonbondedForces(torch.autograd.Function):
        """F(pos, charge, sigma, eps) [N,3] float64, differentiable in charge, sigma and eps
        through the force VJP (force matching).  The position derivative (a Hessian-vector
        product) is not provided: asking for it raises."""

        @staticmethod
        def forward(ctx, pos, charge, sigma, eps, batch: DeviceBatch, params: nb_params):
            b = _rebatch(batch, pos, charge, sigma, eps)
            ws = alloc_workspace(b, params)
            build_cells(b, params, ws)
            force = torch.empty((b.n_atoms, 3), dtype=torch.float64, device=pos.device)
            nonbonded_forces(b, params, ws, force)
            ctx.batch, ctx.params, ctx.ws = b, params, ws
            ctx.dtypes = (charge.dtype, sigma.dtype, eps.dtype)
            return force

        @staticmethod
        def backward(ctx, grad_force):
            if ctx.needs_input_grad[0]:
                raise NotImplementedError("NonbondedForces: no derivative with respect to positions")
            b, params, ws = ctx.batch, ctx.params, ctx.ws
            dev = b.pos.device
            v = grad_force.detach().to(torch.float64).contiguous()
            need = ctx.needs_input_grad
            gq = torch.empty(b.n_atoms, dtype=torch.float64, device=dev) if need[1] else None
            gs = torch.empty(b.sigma.shape[0], dtype=torch.float64, device=dev) if need[2] else None
            ge = torch.empty(b.sigma.shape[0], dtype=torch.float64, device=dev) if need[3] else None
            nonbonded_force_vjp(b, params, ws, v, gq, gs, ge)
            qd, sd, ed = ctx.dtypes
            return (None, None if gq is None else gq.to(qd), None if gs is None else gs.to(sd),
                    None if ge is None else ge.to(ed), None, None)

    return NonbondedEnergy, NonbondedForces


_NE = None
_NF = None


def _functions():
    global _NE, _NF
    if _NE is None:
        _NE, _NF = _autograd()
    return _NE, _NF


def nonbonded_energy_autograd(pos, charge, sigma, eps, batch: DeviceBatch, params: nb_params):
    """Differentiable energies [B] (see NonbondedEnergy)."""
    return _functions()[0].apply(pos, charge, sigma, eps, batch, params)


def nonbonded_forces_autograd(pos, charge, sigma, eps, batch: DeviceBatch, params: nb_params):
    """Forces [N,3] differentiable in charge, sigma and eps (see NonbondedForces)."""
    return _functions()[1].apply(pos, charge, sigma, eps, batch, params)


def __getattr__(name):
    if name == "NonbondedEnergy":
        return _functions()[0]
    if name == "NonbondedForces":
        return _functions()[1]
    raise AttributeError(name)
