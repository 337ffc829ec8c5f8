"""ctypes binding of libdpd.so (include/dpd.h).  Argument marshalling only:
every step of the DPD path runs in the library's HIP kernels.

The library is loaded from this package directory; if it is missing the
import fails loudly (build it with ``python -m paper_1804_06205_amd.build``).
There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EBOX, ERANGE, ESTATE, EBUSY, ECAPACITY = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
PREC_FP64, PREC_MIXED = 0, 1
BOND_HARMONIC, BOND_MORSE_PAPER, BOND_MORSE = 1, 2, 3

_CODE_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENUMERIC: "ENUMERIC",
               EBOX: "EBOX", ERANGE: "ERANGE", ESTATE: "ESTATE", EBUSY: "EBUSY",
               ECAPACITY: "ECAPACITY"}


class DPDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time", ctypes.c_double), ("ke", ctypes.c_double),
                ("kT", ctypes.c_double), ("u_pair", ctypes.c_double),
                ("u_bond", ctypes.c_double), ("w_pair", ctypes.c_double),
                ("w_bond", ctypes.c_double), ("pressure", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("npairs", ctypes.c_int64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("ms_begin", ctypes.c_double), ("ms_fused", ctypes.c_double),
                ("ms_finish", ctypes.c_double), ("n_begin", ctypes.c_int64),
                ("n_fused", ctypes.c_int64), ("n_finish", ctypes.c_int64)]


_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/dpd.h.
SIGNATURES = {
    "dpd_version": (ctypes.c_int, []),
    "dpd_last_error": (ctypes.c_char_p, []),
    "dpd_create": (ctypes.c_int, [ctypes.POINTER(_vp), _d, ctypes.c_int64, _d, _d, _u8,
                                  ctypes.c_int, ctypes.c_uint64, ctypes.c_int, _vp,
                                  ctypes.c_int]),
    "dpd_set_params": (ctypes.c_int, [_vp, _d, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "dpd_add_bonds": (ctypes.c_int, [_vp, ctypes.c_int64, _i32, _i64, _i64, _d, _d, _d]),
    "dpd_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "dpd_step_profiled": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.POINTER(KernelTimes)]),
    "dpd_sync": (ctypes.c_int, [_vp]),
    "dpd_observables": (ctypes.c_int, [_vp, ctypes.POINTER(Obs)]),
    "dpd_get_state": (ctypes.c_int, [_vp, _d, _d, _d, _i64]),
    "dpd_set_state": (ctypes.c_int, [_vp, _d, _d, _d, ctypes.c_int64]),
    "dpd_get_cells": (ctypes.c_int, [_vp, _i64, _i64]),
    "dpd_info": (ctypes.c_int, [_vp, _i64]),
    "dpd_destroy": (None, [_vp]),
    "dpd_variant_count": (ctypes.c_int, []),
    "dpd_variant_shape": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "dpd_set_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dpd_autotune": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]),
    "dpd_pair_noise": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, _d]),
    "dpd_pair_noise_noalloc": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64,
                                              ctypes.POINTER(ctypes.c_uint32),
                                              ctypes.POINTER(ctypes.c_uint32),
                                              ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, _d]),
    "dpd_footprint_bytes": (ctypes.c_int, [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_int, _i64]),
    "dpd_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int64, ctypes.c_int, _vp,
                                        ctypes.c_int]),
    "dpd_batch_admit": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int)]),
    "dpd_batch_advance": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "dpd_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_double)]),
    "dpd_batch_poll": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]),
    "dpd_batch_retire": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dpd_batch_info": (ctypes.c_int, [_vp, _i64]),
    "dpd_batch_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """Loads libdpd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_1804_06205_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def variants() -> list:
    """Shapes {BX, BY, BZ, threads, LDS capacity} of the pair-kernel variants."""
    out = []
    for v in range(lib().dpd_variant_count()):
        a = (ctypes.c_int * 5)()
        _check(lib().dpd_variant_shape(v, a))
        out.append(tuple(a))
    return out


def pair_noise(seed: int, ti, tj, s, precision: str = "mixed") -> np.ndarray:
    """theta_ij(s) as the step kernels compute it, for arrays of triples."""
    u32 = ctypes.POINTER(ctypes.c_uint32)
    ti = np.ascontiguousarray(ti, np.uint32)
    tj = np.ascontiguousarray(tj, np.uint32)
    s = np.ascontiguousarray(np.broadcast_to(s, ti.shape), np.uint32)
    out = np.zeros(ti.shape[0])
    _check(lib().dpd_pair_noise(seed, ti.shape[0], _p(ti, u32), _p(tj, u32), _p(s, u32),
                                PREC_FP64 if precision == "fp64" else PREC_MIXED,
                                _p(out, _d)))
    return out


def pair_noise_noalloc(seed: int, ti, tj, s, precision: str = "mixed") -> np.ndarray:
    """pair_noise through the entry point that allocates no device memory
    (at most 2^18 triples per call)."""
    u32 = ctypes.POINTER(ctypes.c_uint32)
    ti = np.ascontiguousarray(ti, np.uint32)
    tj = np.ascontiguousarray(tj, np.uint32)
    s = np.ascontiguousarray(np.broadcast_to(s, ti.shape), np.uint32)
    out = np.zeros(ti.shape[0])
    _check(lib().dpd_pair_noise_noalloc(seed, ti.shape[0], _p(ti, u32), _p(tj, u32), _p(s, u32),
                                        PREC_FP64 if precision == "fp64" else PREC_MIXED,
                                        _p(out, _d)))
    return out


def footprint_bytes(L, n: int, nbonds: int = 0, precision: str = "mixed",
                    cell_capacity: int = 0) -> int:
    """Device bytes a system of this shape will hold (dpd_info's device_bytes)."""
    Lv = _f64(L, (3,))
    out = ctypes.c_int64()
    _check(lib().dpd_footprint_bytes(_p(Lv, _d), n, nbonds,
                                     PREC_FP64 if precision == "fp64" else PREC_MIXED,
                                     cell_capacity, ctypes.byref(out)))
    return out.value


def last_error() -> str:
    return lib().dpd_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise DPDError(rc, last_error())


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _stream_handle(stream):
    """Accepts None, an int handle or a torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class System:
    """One DPD system on the current GPU (a thin owner of a ``dpd_system*``)."""

    def __init__(self, L, pos, vel, types=None, ntypes: int = 1, seed: int = 0,
                 precision: str = "mixed", stream=None, cell_capacity: int = 0):
        self._h = None
        Lv = _f64(L, (3,))
        pos = _f64(pos, (-1, 3))
        vel = _f64(vel, (-1, 3))
        n = pos.shape[0]
        t = None if types is None else np.ascontiguousarray(types, dtype=np.uint8)
        prec = PREC_FP64 if precision == "fp64" else PREC_MIXED
        h = _vp()
        _check(lib().dpd_create(ctypes.byref(h), _p(Lv, _d), n, _p(pos, _d), _p(vel, _d),
                                None if t is None else _p(t, _u8), ntypes, seed, prec,
                                _stream_handle(stream), cell_capacity))
        self._h = h
        self.n = n
        self.L = Lv
        self.ntypes = ntypes
        self.precision = precision

    @classmethod
    def from_workload(cls, w, precision: str | None = None, stream=None, cell_capacity: int = 0):
        """Creates, parameterises and bonds a system from a workloads.Workload."""
        s = cls(w.L, w.pos, w.vel, w.types, w.ntypes, w.seed, precision or w.precision,
                stream, cell_capacity)
        s.set_params(w.a, w.gamma, w.sigma, w.kT, w.dt, w.lam)
        if w.nbonds:
            s.add_bonds(w.btype, w.bi, w.bj, w.r_e, w.k, w.alpha)
        return s

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.dpd_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, a, gamma, sigma, kT, dt, lam=0.65):
        a = _f64(np.atleast_2d(a))
        _check(lib().dpd_set_params(self._h, _p(a, _d), gamma, sigma, kT, dt, lam))

    def add_bonds(self, btype, bi, bj, r_e, k, alpha):
        bt = np.ascontiguousarray(btype, np.int32)
        bi = np.ascontiguousarray(bi, np.int64)
        bj = np.ascontiguousarray(bj, np.int64)
        r_e, k, alpha = _f64(r_e), _f64(k), _f64(alpha)
        _check(lib().dpd_add_bonds(self._h, bt.shape[0], _p(bt, _i32), _p(bi, _i64),
                                   _p(bj, _i64), _p(r_e, _d), _p(k, _d), _p(alpha, _d)))

    def step(self, nsteps: int = 1):
        _check(lib().dpd_step(self._h, nsteps))

    def step_profiled(self, nsteps: int) -> dict:
        t = KernelTimes()
        _check(lib().dpd_step_profiled(self._h, nsteps, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in KernelTimes._fields_}

    def sync(self):
        _check(lib().dpd_sync(self._h))

    def observables(self) -> dict:
        o = Obs()
        _check(lib().dpd_observables(self._h, ctypes.byref(o)))
        d = {f: getattr(o, f) for f, _ in Obs._fields_}
        d["momentum"] = list(o.momentum)
        return d

    def get_state(self, force: bool = True):
        pos = np.zeros((self.n, 3))
        vel = np.zeros((self.n, 3))
        frc = np.zeros((self.n, 3)) if force else None
        step = ctypes.c_int64()
        _check(lib().dpd_get_state(self._h, _p(pos, _d), _p(vel, _d),
                                   None if frc is None else _p(frc, _d), ctypes.byref(step)))
        return pos, vel, frc, step.value

    def set_state(self, pos, vel, force=None, step: int = 0):
        pos = _f64(pos, (-1, 3))
        vel = _f64(vel, (-1, 3))
        f = None if force is None else _f64(force, (-1, 3))
        _check(lib().dpd_set_state(self._h, _p(pos, _d), _p(vel, _d),
                                   None if f is None else _p(f, _d), step))

    def get_cells(self):
        info = self.info()
        cell = np.zeros(self.n, np.int64)
        count = np.zeros(info["ncells"], np.int64)
        _check(lib().dpd_get_cells(self._h, _p(cell, _i64), _p(count, _i64)))
        return cell, count

    def set_variant(self, variant: int):
        _check(lib().dpd_set_variant(self._h, variant))

    def autotune(self, trials: int = 3):
        """Times every brick variant on the current state; keeps the fastest."""
        v = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().dpd_autotune(self._h, trials, ctypes.byref(v), ctypes.byref(ms)))
        return v.value, ms.value

    def info(self) -> dict:
        out = np.zeros(8, np.int64)
        _check(lib().dpd_info(self._h, _p(out, _i64)))
        keys = ("n", "ncells", "cell_capacity", "device_bytes", "nx", "ny", "nz", "precision")
        return dict(zip(keys, (int(v) for v in out)))


class Batch:
    """A replica batch (dpd_batch_*): resident systems advanced together, one
    captured HIP graph per window of K steps."""

    def __init__(self, budget_bytes: int, max_replicas: int = 1024, stream=None,
                 variant: int = -1):
        self._h = None
        h = _vp()
        _check(lib().dpd_batch_create(ctypes.byref(h), int(budget_bytes), max_replicas,
                                      _stream_handle(stream), variant))
        self._h = h
        self.max_replicas = max_replicas
        self._members = {}      # slot -> System (keeps them alive while resident)

    def admit(self, system: System, nsteps: int) -> int:
        slot = ctypes.c_int()
        _check(lib().dpd_batch_admit(self._h, system._h, nsteps, ctypes.byref(slot)))
        self._members[slot.value] = system
        return slot.value

    def advance(self, K: int):
        _check(lib().dpd_batch_advance(self._h, K))

    def autotune(self, K: int = 20):
        """One K-step window with each brick variant; keeps the fastest.
        Returns (variant, ms per step)."""
        v = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().dpd_batch_autotune(self._h, K, ctypes.byref(v), ctypes.byref(ms)))
        return v.value, ms.value

    def poll(self) -> list:
        """Waits for the enqueued windows; slots that finished since the last poll."""
        out = (ctypes.c_int * self.max_replicas)()
        nd = ctypes.c_int()
        _check(lib().dpd_batch_poll(self._h, out, self.max_replicas, ctypes.byref(nd)))
        return list(out[:nd.value])

    def retire(self, slot: int) -> System:
        _check(lib().dpd_batch_retire(self._h, slot))
        return self._members.pop(slot)

    def info(self) -> dict:
        out = np.zeros(6, np.int64)
        _check(lib().dpd_batch_info(self._h, _p(out, _i64)))
        keys = ("resident", "bytes_used", "budget", "captures", "windows", "variant")
        return dict(zip(keys, (int(v) for v in out)))

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.dpd_batch_destroy(self._h)
        self._h = None
        self._members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
