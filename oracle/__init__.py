"""Python shim over the FP64 DPD oracle (``oracle/dpd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1804_06205_amd``) and neither imports the other;
the seeded inputs both consume come from ``paper_1804_06205_amd.workloads``,
which holds none of the method's arithmetic.

Each wrapper names the passage of the paper (arXiv 1804.06205) that the C
function follows; the C source states the formulas.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpd_oracle.cpp")
_LIB = os.environ.get("DPD_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u32 = ctypes.POINTER(ctypes.c_uint32)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_philox4x32_10.argtypes = [_u32, _u32, _u32]
        L.oracle_philox4x32_10.restype = None
        L.oracle_pair_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint64]
        L.oracle_pair_noise.restype = ctypes.c_double
        L.oracle_pair_noise_batch.argtypes = [ctypes.c_uint64, ctypes.c_int64, _u32, _u32,
                                              ctypes.POINTER(ctypes.c_uint64), _d]
        L.oracle_pair_noise_batch.restype = None
        L.oracle_wrap.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_wrap.restype = ctypes.c_double
        L.oracle_bond_term.argtypes = [ctypes.c_int, _d, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _d, _d, _d]
        L.oracle_bond_term.restype = ctypes.c_int
        L.oracle_bin.argtypes = [ctypes.c_int64, _d, _d, _i64, _i64, _i64, _i64]
        L.oracle_bin.restype = None
        pf = [ctypes.c_int64, _d, _d, _d, _u8, ctypes.c_int, _d, ctypes.c_double,
              ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, _d, _d]
        L.oracle_pair_forces.argtypes = pf
        L.oracle_pair_forces.restype = None
        L.oracle_pair_forces_brute.argtypes = pf
        L.oracle_pair_forces_brute.restype = None
        L.oracle_bond_forces.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_int64, _i32, _i64,
                                         _i64, _d, _d, _d, _d, _d]
        L.oracle_bond_forces.restype = ctypes.c_int
        L.oracle_forces.argtypes = [ctypes.c_int64, _d, _d, _d, _u8, ctypes.c_int, _d, _d,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, _i32,
                                    _i64, _i64, _d, _d, _d, _d]
        L.oracle_forces.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _u8, ctypes.c_int, _d, _d,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, _i32, _i64, _i64, _d, _d, _d]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_observables.argtypes = [ctypes.c_int64, _d, _d, _d, _u8, ctypes.c_int, _d,
                                         ctypes.c_int64, _i32, _i64, _i64, _d, _d, _d, _d]
        L.oracle_observables.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def philox4x32_10(ctr, key) -> np.ndarray:
    """Raw Philox4x32-10 words for one counter (4 x u32) and key (2 x u32)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c, _u32), _p(k, _u32), _p(out, _u32))
    return out


def pair_noise(seed: int, ti: int, tj: int, s: int) -> float:
    """theta_ij(s), the standard normal of the random force (text after Eq. 5)."""
    return lib().oracle_pair_noise(seed, ti, tj, s)


def pair_noise_batch(seed: int, ti, tj, s) -> np.ndarray:
    """theta for arrays of (tag_i, tag_j, s)."""
    ti = np.ascontiguousarray(ti, dtype=np.uint32)
    tj = np.ascontiguousarray(tj, dtype=np.uint32)
    s = np.ascontiguousarray(np.broadcast_to(s, ti.shape), dtype=np.uint64)
    out = np.zeros(ti.shape[0])
    lib().oracle_pair_noise_batch(seed, ti.shape[0], _p(ti, _u32), _p(tj, _u32),
                                  _p(s, ctypes.POINTER(ctypes.c_uint64)), _p(out, _d))
    return out


def wrap(x: float, L: float) -> float:
    """Periodic wrap of one coordinate ("boundary_check", Fig. 1)."""
    return lib().oracle_wrap(x, L)


def bond_term(btype: int, d, r_e: float, k: float, alpha: float):
    """Force on i, energy and virial of one bond record (Eqs. 6-8, Fig. 3a)."""
    d = _f64(d, (3,))
    F = np.zeros(3)
    U = ctypes.c_double()
    W = ctypes.c_double()
    rc = lib().oracle_bond_term(btype, _p(d, _d), r_e, k, alpha, _p(F, _d), ctypes.byref(U),
                                ctypes.byref(W))
    if rc != 0:
        raise ValueError("bad bond type")
    return F, U.value, W.value


def bin_cells(pos, L):
    """Per-step cell list (design section, Fig. 1 step 3): per-particle cell
    coordinates, per-cell counts, exclusive starts and the (cell, tag) order."""
    pos = _f64(pos)
    Lv = _f64(L, (3,))
    n = pos.shape[0]
    nc = np.floor(Lv).astype(np.int64)
    ncells = int(nc.prod())
    cxyz = np.zeros((n, 3), np.int64)
    count = np.zeros(ncells, np.int64)
    start = np.zeros(ncells + 1, np.int64)
    order = np.zeros(n, np.int64)
    lib().oracle_bin(n, _p(Lv, _d), _p(pos, _d), _p(cxyz, _i64), _p(count, _i64),
                     _p(start, _i64), _p(order, _i64))
    return cxyz, count, start, order


def _types(types, n):
    if types is None:
        return np.zeros(n, np.uint8)
    return np.ascontiguousarray(types, dtype=np.uint8)


def pair_forces(pos, vt, L, a, gamma, sigma, dt, seed, s, types=None, brute=False):
    """F^C + F^D + F^R on every particle (Eqs. 3-4) at noise counter s.
    Returns (F, U_pair, W_pair, npairs)."""
    pos = _f64(pos)
    vt = _f64(vt)
    n = pos.shape[0]
    Lv = _f64(L, (3,))
    a = _f64(np.atleast_2d(a))
    t = _types(types, n)
    F = np.zeros((n, 3))
    out = np.zeros(3)
    fn = lib().oracle_pair_forces_brute if brute else lib().oracle_pair_forces
    fn(n, _p(Lv, _d), _p(pos, _d), _p(vt, _d), _p(t, _u8), a.shape[0], _p(a, _d), gamma,
       sigma, dt, seed, s, _p(F, _d), _p(out, _d))
    return F, out[0], out[1], int(round(out[2]))


def _bond_args(bonds, ):
    if bonds is None or len(bonds["btype"]) == 0:
        z = np.zeros(1)
        return (0, np.zeros(1, np.int32), np.zeros(1, np.int64), np.zeros(1, np.int64), z, z, z)
    return (len(bonds["btype"]), np.ascontiguousarray(bonds["btype"], np.int32),
            np.ascontiguousarray(bonds["bi"], np.int64),
            np.ascontiguousarray(bonds["bj"], np.int64), _f64(bonds["r_e"]), _f64(bonds["k"]),
            _f64(bonds["alpha"]))


def bond_forces(pos, L, bonds):
    """F^S over the bond list (Eq. 8).  Returns (F, U_bond, W_bond)."""
    pos = _f64(pos)
    n = pos.shape[0]
    Lv = _f64(L, (3,))
    nb, bt, bi, bj, re, kk, al = _bond_args(bonds)
    F = np.zeros((n, 3))
    out = np.zeros(2)
    rc = lib().oracle_bond_forces(n, _p(Lv, _d), _p(pos, _d), nb, _p(bt, _i32), _p(bi, _i64),
                                  _p(bj, _i64), _p(re, _d), _p(kk, _d), _p(al, _d), _p(F, _d),
                                  _p(out, _d))
    if rc != 0:
        raise ValueError("bad bond record")
    return F, out[0], out[1]


def _sp(params):
    return np.array([params["gamma"], params["sigma"], params["dt"], params["lam"]], np.float64)


def forces(pos, vt, L, types, params, seed, s, bonds=None):
    """Total force F_pair(x, vt; s) + F_bond(x); the initial force of a run is
    this with vt = v and s = 0."""
    pos = _f64(pos)
    vt = _f64(vt)
    n = pos.shape[0]
    Lv = _f64(L, (3,))
    a = _f64(np.atleast_2d(params["a"]))
    t = _types(types, n)
    sp = _sp(params)
    nb, bt, bi, bj, re, kk, al = _bond_args(bonds)
    F = np.zeros((n, 3))
    rc = lib().oracle_forces(n, _p(Lv, _d), _p(pos, _d), _p(vt, _d), _p(t, _u8), a.shape[0],
                             _p(a, _d), _p(sp, _d), seed, s, nb, _p(bt, _i32), _p(bi, _i64),
                             _p(bj, _i64), _p(re, _d), _p(kk, _d), _p(al, _d), _p(F, _d))
    if rc != 0:
        raise ValueError("bad bond record")
    return F


class State:
    """An oracle trajectory: (pos, vel, force) in tag order plus the step counter."""

    def __init__(self, pos, vel, L, types, params, seed, bonds=None, force=None, step=0):
        self.pos = _f64(pos).copy()
        self.vel = _f64(vel).copy()
        self.L = _f64(L, (3,)).copy()
        self.types = _types(types, self.pos.shape[0]).copy()
        self.params = dict(params)
        self.a = _f64(np.atleast_2d(params["a"])).copy()
        self.seed = int(seed)
        self.bonds = bonds
        self.step_count = int(step)
        if force is None:
            force = forces(self.pos, self.vel, self.L, self.types, self.params, self.seed,
                           self.step_count, bonds)
        self.force = _f64(force).copy()

    @classmethod
    def from_workload(cls, w):
        return cls(w.pos, w.vel, w.L, w.types, w.params(), w.seed, w.bonds())

    def step(self, nsteps: int = 1) -> "State":
        """Advance by nsteps (Fig. 1 with Groot's modified velocity Verlet)."""
        n = self.pos.shape[0]
        nb, bt, bi, bj, re, kk, al = _bond_args(self.bonds)
        sp = _sp(self.params)
        rc = lib().oracle_run(n, _p(self.L, _d), _p(self.pos, _d), _p(self.vel, _d),
                              _p(self.force, _d), _p(self.types, _u8), self.a.shape[0],
                              _p(self.a, _d), _p(sp, _d), self.seed, self.step_count, nsteps,
                              nb, _p(bt, _i32), _p(bi, _i64), _p(bj, _i64), _p(re, _d),
                              _p(kk, _d), _p(al, _d))
        if rc == -2:
            raise FloatingPointError("displacement above half a box")
        if rc != 0:
            raise ValueError("bad bond record")
        self.step_count += nsteps
        return self

    def observables(self) -> dict:
        return observables(self.pos, self.vel, self.L, self.types, self.a, self.bonds)


OBS_KEYS = ("ke", "kT", "u_pair", "u_bond", "w_pair", "w_bond", "pressure", "px", "py", "pz",
            "npairs", "e_total", "virial", "volume")


def observables(pos, vel, L, types, a, bonds=None) -> dict:
    """KE, kT = 2KE/(3N-3), pair and bond energies (Fig. 3a accumulates Ebond),
    virial pressure p = (2KE + W)/(3V), momentum, in-range pair count."""
    pos = _f64(pos)
    vel = _f64(vel)
    n = pos.shape[0]
    Lv = _f64(L, (3,))
    a = _f64(np.atleast_2d(a))
    t = _types(types, n)
    nb, bt, bi, bj, re, kk, al = _bond_args(bonds)
    out = np.zeros(14)
    rc = lib().oracle_observables(n, _p(Lv, _d), _p(pos, _d), _p(vel, _d), _p(t, _u8),
                                  a.shape[0], _p(a, _d), nb, _p(bt, _i32), _p(bi, _i64),
                                  _p(bj, _i64), _p(re, _d), _p(kk, _d), _p(al, _d), _p(out, _d))
    if rc != 0:
        raise ValueError("bad bond record")
    d = dict(zip(OBS_KEYS, out.tolist()))
    d["npairs"] = int(round(d["npairs"]))
    return d
