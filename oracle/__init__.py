"""FP64 CPU oracle for LJ + ATM forces and the r-RESPA loop (ctypes over oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with
the HIP library; the two meet only through the seeded inputs of
``paper_2507_11172_amd.workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

from . import build as _build

_LIB = None

OK = 0
ERR_INVALID_ARG = -1
ERR_BOX_TOO_SMALL = -2
ERR_NOT_MULTIPLE_OF_K = -3
ERR_NONFINITE = -5
ERR_OOM = -7


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("oracle %s failed with status %d" % (what, code))
        self.code = code


class _MD(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double), ("rc_pair", C.c_double),
                ("nu", C.c_double), ("rc3", C.c_double), ("mass", C.c_double),
                ("dt", C.c_double), ("shift", C.c_int), ("nthreads", C.c_int)]


_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        L.orc_wrap.argtypes = [C.c_int64, _D, _D, _D]
        L.orc_cell_index.argtypes = [C.c_int64, _D, _D, _I32, _I32]
        L.orc_pair.argtypes = [C.c_int64, _D, _D, C.c_double, C.c_double, C.c_double, C.c_int,
                               _D, _D, _I64, C.c_int]
        L.orc_triplet.argtypes = [C.c_int64, _D, _D, C.c_double, C.c_double, _D, _D, _I64, C.c_int]
        L.orc_triplet_class.argtypes = [C.c_int64, _D, _D, C.c_double, C.c_double, C.c_double,
                                        _D, _D, _I64, C.c_int]
        L.orc_respa_nested.argtypes = [C.c_int64, _D, _D, _D, C.POINTER(_MD), C.c_int64, C.c_int,
                                       C.c_int, C.c_double, _D]
        L.orc_respa_alg1.argtypes = [C.c_int64, _D, _D, _D, C.POINTER(_MD), C.c_int64, C.c_int, _D]
        L.orc_triplet_list.argtypes = [C.c_int64, _D, _D, C.c_double, _I32, C.c_int64]
        L.orc_triplet_list.restype = C.c_int64
        L.orc_subset.argtypes = [C.c_int64, _D, _D, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_int64, _I64, _D, _D, _I64, C.c_int]
        L.orc_respa.argtypes = [C.c_int64, _D, _D, _D, C.POINTER(_MD), C.c_int64, C.c_int, _D]
        L.orc_vv.argtypes = [C.c_int64, _D, _D, _D, C.POINTER(_MD), C.c_int64, _D]
        L.orc_atm_energy.argtypes = [_D, _D, C.c_double]
        L.orc_atm_energy.restype = C.c_double
        L.orc_atm_forces.argtypes = [_D, _D, C.c_double, _D]
        L.orc_lj.argtypes = [C.c_double, C.c_double, C.c_double, _D]
        L.orc_lj.restype = C.c_double
        _LIB = L
    return _LIB


def _d(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def wrap(x, box) -> np.ndarray:
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    out = np.empty_like(x)
    lib().orc_wrap(x.shape[0], _d(x), _d(box), _d(out))
    return out


def cell_index(x, box, n_cells) -> np.ndarray:
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    nc = np.ascontiguousarray(np.asarray(n_cells, dtype=np.int32).reshape(3))
    out = np.empty(x.shape[0], dtype=np.int32)
    _check(lib().orc_cell_index(x.shape[0], _d(x), _d(box), nc.ctypes.data_as(_I32),
                                out.ctypes.data_as(_I32)), "cell_index")
    return out


@dataclass
class ForceResult:
    f: np.ndarray      # [N, 3]
    energy: float      # U
    virial: float      # W = sum x . F
    count: int         # interacting pairs or triplets


def pair_forces(x, box, eps=1.0, sigma=1.0, rc=2.5, shift=True, nthreads=0) -> ForceResult:
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    f = np.empty_like(x)
    uw = np.zeros(2)
    cnt = C.c_int64(0)
    _check(lib().orc_pair(x.shape[0], _d(x), _d(box), eps, sigma, rc, int(bool(shift)), _d(f),
                          _d(uw), C.byref(cnt), nthreads), "pair_forces")
    return ForceResult(f, float(uw[0]), float(uw[1]), int(cnt.value))


def triplet_forces(x, box, nu=0.073, rc=2.5, r_lo=0.0, nthreads=0) -> ForceResult:
    """ATM over the triplets with all three edges <= rc; with r_lo > 0 only those whose
    longest edge exceeds r_lo (the outer distance class (r_lo, rc])."""
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    f = np.empty_like(x)
    uw = np.zeros(2)
    cnt = C.c_int64(0)
    _check(lib().orc_triplet_class(x.shape[0], _d(x), _d(box), nu, r_lo, rc, _d(f), _d(uw),
                                   C.byref(cnt), nthreads), "triplet_forces")
    return ForceResult(f, float(uw[0]), float(uw[1]), int(cnt.value))


def triplet_list(x, box, rc=2.5) -> np.ndarray:
    """All interacting triplets as an [M, 3] int32 array of (i<j<k), lexicographic."""
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    n = lib().orc_triplet_list(x.shape[0], _d(x), _d(box), rc, None, 0)
    if n < 0:
        raise OracleError(int(n), "triplet_list")
    out = np.zeros((max(n, 1), 3), dtype=np.int32)
    n2 = lib().orc_triplet_list(x.shape[0], _d(x), _d(box), rc, out.ctypes.data_as(_I32), n)
    assert n2 == n
    return out[:n]


def subset_forces(x, box, idx, eps=1.0, sigma=1.0, rc_pair=2.5, nu=0.073, rc3=2.5,
                  nthreads=0, counts=False):
    """Exact (F2, F3) on the chosen particles of an arbitrarily large system; with
    counts=True also (pairs, triplets) summed over the chosen particles (each pair or
    triplet once per chosen member)."""
    x = _f64(x).reshape(-1, 3)
    box = _f64(box).reshape(3)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    f2 = np.empty((idx.shape[0], 3))
    f3 = np.empty((idx.shape[0], 3))
    cnt = np.zeros(2, dtype=np.int64)
    _check(lib().orc_subset(x.shape[0], _d(x), _d(box), eps, sigma, rc_pair, nu, rc3,
                            idx.shape[0], idx.ctypes.data_as(_I64), _d(f2), _d(f3),
                            cnt.ctypes.data_as(_I64), nthreads),
           "subset_forces")
    if counts:
        return f2, f3, (int(cnt[0]), int(cnt[1]))
    return f2, f3


def _md(eps, sigma, rc_pair, nu, rc3, mass, dt, shift, nthreads) -> _MD:
    return _MD(eps, sigma, rc_pair, nu, rc3, mass, dt, int(bool(shift)), nthreads)


def respa(x, v, box, n_iter, k, eps=1.0, sigma=1.0, rc_pair=2.5, nu=0.073, rc3=2.5, mass=1.0,
          dt=0.001, shift=True, nthreads=0):
    """Runs Algorithm 2 on copies; returns (x, v, e_full[n_iter/k + 1, 5])."""
    x = _f64(x).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    box = _f64(box).reshape(3)
    e = np.zeros((n_iter // k + 1 if k > 0 else 1, 5))
    p = _md(eps, sigma, rc_pair, nu, rc3, mass, dt, shift, nthreads)
    _check(lib().orc_respa(x.shape[0], _d(x), _d(v), _d(box), C.byref(p), n_iter, k, _d(e)),
           "respa")
    return x, v, e


def respa_nested(x, v, box, n_iter, k, k_outer, r_a, eps=1.0, sigma=1.0, rc_pair=2.5,
                 nu=0.073, rc3=2.5, mass=1.0, dt=0.001, shift=True, nthreads=0):
    """Three-level r-RESPA over the triplet distance classes split at r_a: F2 every step,
    the inner class every k steps, the outer class every k * k_outer steps.  Returns
    (x, v, e_full[n_iter / (k k_outer) + 1, 5])."""
    x = _f64(x).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    box = _f64(box).reshape(3)
    span = k * k_outer
    e = np.zeros((n_iter // span + 1 if span > 0 else 1, 5))
    p = _md(eps, sigma, rc_pair, nu, rc3, mass, dt, shift, nthreads)
    _check(lib().orc_respa_nested(x.shape[0], _d(x), _d(v), _d(box), C.byref(p), n_iter, k,
                                  k_outer, r_a, _d(e)), "respa_nested")
    return x, v, e


def respa_alg1(x, v, box, n_outer, P, eps=1.0, sigma=1.0, rc_pair=2.5, nu=0.073, rc3=2.5,
               mass=1.0, delta_t=0.004, shift=True, nthreads=0):
    """Algorithm 1 as printed: full steps delta_t, F2 over P sub-steps, F3 kicks per full
    step.  Returns (x, v, e[n_outer + 1, 5])."""
    x = _f64(x).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    box = _f64(box).reshape(3)
    e = np.zeros((n_outer + 1, 5))
    p = _md(eps, sigma, rc_pair, nu, rc3, mass, delta_t, shift, nthreads)
    _check(lib().orc_respa_alg1(x.shape[0], _d(x), _d(v), _d(box), C.byref(p), n_outer, P, _d(e)),
           "respa_alg1")
    return x, v, e


def velocity_verlet(x, v, box, n_iter, eps=1.0, sigma=1.0, rc_pair=2.5, nu=0.073, rc3=2.5,
                    mass=1.0, dt=0.001, shift=True, nthreads=0):
    """Textbook velocity Verlet with F2 + F3 every step; returns (x, v, e[n_iter + 1, 5])."""
    x = _f64(x).reshape(-1, 3).copy()
    v = _f64(v).reshape(-1, 3).copy()
    box = _f64(box).reshape(3)
    e = np.zeros((n_iter + 1, 5))
    p = _md(eps, sigma, rc_pair, nu, rc3, mass, dt, shift, nthreads)
    _check(lib().orc_vv(x.shape[0], _d(x), _d(v), _d(box), C.byref(p), n_iter, _d(e)), "vv")
    return x, v, e


def atm_energy(u, w, nu=0.073) -> float:
    """phi3 of one triplet from its edge vectors u = x_j - x_i and w = x_k - x_i."""
    u = _f64(u).reshape(3)
    w = _f64(w).reshape(3)
    return float(lib().orc_atm_energy(_d(u), _d(w), nu))


def atm_forces(u, w, nu=0.073) -> np.ndarray:
    """[3, 3] forces on (i, j, k) of one triplet."""
    u = _f64(u).reshape(3)
    w = _f64(w).reshape(3)
    out = np.zeros(9)
    lib().orc_atm_forces(_d(u), _d(w), nu, _d(out))
    return out.reshape(3, 3)


def lj(r2, eps=1.0, sigma=1.0) -> Tuple[float, float]:
    """(phi2, fr) with F_j = fr * d for d = x_j - x_i."""
    fr = C.c_double(0.0)
    e = lib().orc_lj(float(r2), eps, sigma, C.byref(fr))
    return float(e), float(fr.value)


def rvite(total_energy: np.ndarray, kinetic: np.ndarray) -> float:
    """Relative Variation In True Energy (Sec. 4.2, Eq. 4): mean |e - mean(e)| / mean(K)."""
    e = np.asarray(total_energy, dtype=np.float64)
    k = float(np.mean(kinetic))
    return float(np.mean(np.abs(e - e.mean())) / k)


def num_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
