"""FP64 CPU oracle for the short-range nonbonded hot path (ctypes wrapper of nb_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the GPU library never does.  It shares no
code with the GPU library.

The definitions it evaluates are written out in ``nb_oracle.c`` (ACEMD paper,
section 3: cutoff Lennard-Jones plus electrostatics with bonded exclusions, the
electrostatics being the real-space part of the Ewald/PME split).  Parameter
gradients follow from the per-atom partial sums the C code returns:

    dE/dq_i     = phi_i
    dE/dsigma_t = sum_{i: t_i = t} a_i
    dE/deps_t   = (1/eps_t) sum_{i: t_i = t} b_i      (0 where eps_t = 0: the derivative
                                                     of sqrt(eps_t eps_j) is unbounded there)
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nb_oracle.c")
_LIB = os.path.join(_HERE, "libnb_oracle.so")

# Coulomb constant e^2 N_A / (4 pi eps0) in kJ mol^-1 A e^-2, from the CODATA 2018
# exact values of e and N_A and the recommended eps0.
_E = 1.602176634e-19
_NA = 6.02214076e23
_EPS0 = 8.8541878128e-12
COULOMB_K = _E * _E / (4.0 * np.pi * _EPS0) * 1e10 * _NA / 1e3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (OpenMP, -O2, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.nbo_rows.restype = ctypes.c_int
        lib.nbo_rows.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, P, P, P,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.nbo_ewald_corrections.restype = ctypes.c_int
        lib.nbo_ewald_corrections.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                                              ctypes.c_double, P, P, P, P, P]
        D = ctypes.c_double
        lib.nbo_rows_vjp.restype = ctypes.c_int
        lib.nbo_rows_vjp.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, P, P, P, D, D, D,
                                     P, P, D, D, D, P,
                                     ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.nbo_rows_ff.restype = ctypes.c_int
        lib.nbo_rows_ff.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, P, P, P, D, D, D,
                                    P, P, D, D, D,
                                    ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.nbo_ewald_corrections_ff.restype = ctypes.c_int
        lib.nbo_ewald_corrections_ff.argtypes = [ctypes.c_int64, P, P, P, P, P, P, D, P, D, D, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(off, idx):
    """Contiguous int32 CSR arrays (a placeholder entry for an empty index list)."""
    o = np.ascontiguousarray(off, np.int32)
    i = np.ascontiguousarray(idx, np.int32)
    return o, (i if i.size else np.zeros(1, np.int32))


def evaluate(pos, charge, types, sigma, eps, excl_offset, excl_index, box, cutoff, beta,
             ke: float = COULOMB_K, rows: Optional[np.ndarray] = None, nthreads: int = 0,
             pair14_offset=None, pair14_index=None, scale14_lj: float = 1.0, scale14_coul: float = 1.0,
             lj_switch_on: float = 0.0, vjp=None) -> dict:
    """Evaluate the brute-force sums for every atom (rows=None) or for the atoms in ``rows``.

    Inputs are promoted to float64; pass exactly the values the device computes with.
    Returns per-row arrays (force [m,3], energy [m], phi [m], a_sig [m], b_eps [m]) and
    totals over the evaluated rows (virial [3,3], e_lj, e_c, energy_total, pairs).  With
    rows=None also the per-type gradients dsigma [T] and deps [T].

    Force-field options: pairs in the 1-4 lists (CSR, union of both rows, not excluded)
    have their LJ term scaled by scale14_lj and their Coulomb term by scale14_coul; with
    lj_switch_on = r_on > 0 the LJ term is switched off between r_on and the cutoff.

    vjp: a vector v [N,3]; then also the derivatives of L = sum_i v_i . F_i with respect to
    the parameters (force matching): vjp_charge [m] per row, and with rows=None
    vjp_sigma [T] and vjp_eps [T] (0 for eps_t = 0).
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    q = np.ascontiguousarray(charge, np.float64)
    t = np.ascontiguousarray(types, np.int32)
    sig = np.ascontiguousarray(sigma, np.float64)
    ep = np.ascontiguousarray(eps, np.float64)
    eo = np.ascontiguousarray(excl_offset, np.int32)
    ei = np.ascontiguousarray(excl_index, np.int32)
    if ei.size == 0:
        ei = np.zeros(1, np.int32)
    bx = np.ascontiguousarray(box, np.float64).reshape(3)
    r = None if rows is None else np.ascontiguousarray(rows, np.int64)
    m = n if r is None else r.shape[0]
    force = np.zeros((m, 3))
    energy = np.zeros(m)
    phi = np.zeros(m)
    a_sig = np.zeros(m)
    b_eps = np.zeros(m)
    vir = np.zeros(9)
    e_lj = ctypes.c_double()
    e_c = ctypes.c_double()
    npairs = ctypes.c_int64()
    po, pi = _csr(pair14_offset, pair14_index) if pair14_offset is not None else (None, None)
    vv = None if vjp is None else np.ascontiguousarray(vjp, np.float64).reshape(n, 3)
    dq2 = np.zeros(m) if vv is not None else None
    a2 = np.zeros(m) if vv is not None else None
    b2 = np.zeros(m) if vv is not None else None
    rc = lib.nbo_rows_vjp(n, _ptr(pos), _ptr(q), _ptr(t), int(sig.shape[0]), _ptr(sig), _ptr(ep),
                          _ptr(eo), _ptr(ei), _ptr(bx), float(cutoff), float(beta), float(ke),
                          _ptr(po), _ptr(pi), float(scale14_lj), float(scale14_coul), float(lj_switch_on),
                          _ptr(vv), m, _ptr(r), _ptr(force), _ptr(energy), _ptr(phi), _ptr(a_sig), _ptr(b_eps),
                          _ptr(dq2), _ptr(a2), _ptr(b2),
                          _ptr(vir), ctypes.byref(e_lj), ctypes.byref(e_c), ctypes.byref(npairs),
                          int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    out = dict(force=force, energy=energy, phi=phi, a_sig=a_sig, b_eps=b_eps,
               virial=vir.reshape(3, 3), e_lj=e_lj.value, e_c=e_c.value,
               energy_total=e_lj.value + e_c.value, pairs=int(npairs.value))
    if r is None:
        T = sig.shape[0]
        dsig = np.zeros(T)
        bsum = np.zeros(T)
        np.add.at(dsig, t, a_sig)
        np.add.at(bsum, t, b_eps)
        deps = np.where(ep > 0, bsum / np.where(ep > 0, ep, 1.0), 0.0)
        out.update(dsigma=dsig, deps=deps)
    if vv is not None:
        out["vjp_charge"] = dq2
        if r is None:
            T = sig.shape[0]
            vs = np.zeros(T)
            vb = np.zeros(T)
            np.add.at(vs, t, a2)
            np.add.at(vb, t, b2)
            out.update(vjp_sigma=vs, vjp_eps=np.where(ep > 0, vb / np.where(ep > 0, ep, 1.0), 0.0))
    return out


def evaluate_system(system, rows=None, nthreads: int = 0, ke: float = COULOMB_K, **ff) -> dict:
    """``evaluate`` on an object with the fields of ``systems.System`` (its 1-4 lists, when
    it has them, and the force-field options given as keyword arguments)."""
    if getattr(system, "pair14_offset", None) is not None and "pair14_offset" not in ff:
        ff = dict(ff, pair14_offset=system.pair14_offset, pair14_index=system.pair14_index)
    return evaluate(system.pos, system.charge, system.type, system.sigma, system.eps,
                    system.excl_offset, system.excl_index, system.box, system.cutoff,
                    system.beta, ke=ke, rows=rows, nthreads=nthreads, **ff)


def ewald_corrections(pos, charge, excl_offset, excl_index, box, beta, ke: float = COULOMB_K,
                      pair14_offset=None, pair14_index=None, scale14_coul: float = 1.0) -> dict:
    """The excluded-pair and self corrections of the Ewald sum (``nbo_ewald_corrections_ff``).

    Inputs are promoted to float64; pass exactly the values the device computes with.
    Returns force [N,3] (of the excluded-pair term), energy [N] (per-atom split: half of
    each excluded pair's term plus the atom's self term), virial [3,3], e_excl, e_self and
    energy_total = e_excl + e_self.  Scaled 1-4 pairs (not excluded) add the excluded-pair
    term times (1 - scale14_coul).
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    q = np.ascontiguousarray(charge, np.float64)
    eo = np.ascontiguousarray(excl_offset, np.int32)
    ei = np.ascontiguousarray(excl_index, np.int32)
    if ei.size == 0:
        ei = np.zeros(1, np.int32)
    bx = np.ascontiguousarray(box, np.float64).reshape(3)
    force = np.zeros((n, 3))
    energy = np.zeros(n)
    vir = np.zeros(9)
    e_excl = ctypes.c_double()
    e_self = ctypes.c_double()
    po, pi = _csr(pair14_offset, pair14_index) if pair14_offset is not None else (None, None)
    rc = lib.nbo_ewald_corrections_ff(n, _ptr(pos), _ptr(q), _ptr(eo), _ptr(ei), _ptr(po), _ptr(pi),
                                      float(scale14_coul), _ptr(bx), float(beta), float(ke), _ptr(force),
                                      _ptr(energy), _ptr(vir), ctypes.byref(e_excl), ctypes.byref(e_self))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return dict(force=force, energy=energy, virial=vir.reshape(3, 3), e_excl=e_excl.value,
                e_self=e_self.value, energy_total=e_excl.value + e_self.value)


def ewald_corrections_system(system, ke: float = COULOMB_K, **ff) -> dict:
    """``ewald_corrections`` on an object with the fields of ``systems.System`` (its 1-4
    lists, when it has them; scale14_coul as a keyword argument)."""
    if getattr(system, "pair14_offset", None) is not None and "pair14_offset" not in ff:
        ff = dict(ff, pair14_offset=system.pair14_offset, pair14_index=system.pair14_index)
    return ewald_corrections(system.pos, system.charge, system.excl_offset, system.excl_index,
                             system.box, system.beta, ke=ke, **ff)
