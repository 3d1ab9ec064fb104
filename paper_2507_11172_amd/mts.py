"""ctypes binding of libmts.so (the C ABI in include/mts.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the
library.  Device arrays are torch tensors on the ROCm device (float64, contiguous,
[N, 3]); the stream is torch's current HIP stream unless one is given.  There is no
CPU fallback: if the library is not built, importing a System raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmts.so")

MTS_OK = 0
MTS_ERR_INVALID_ARG = -1
MTS_ERR_BOX_TOO_SMALL = -2
MTS_ERR_NOT_MULTIPLE_OF_K = -3
MTS_ERR_CAPACITY = -4
MTS_ERR_NONFINITE = -5
MTS_ERR_HIP = -6
MTS_ERR_OOM = -7
MTS_ERR_UNSUPPORTED = -8
MTS_FP64 = 0
MTS_FP32 = 1
MTS_CUTOFF = 0
MTS_DIRECT = 1
MTS_NE = 5

EXPORTS = ("mts_init_system", "mts_destroy_system", "mts_build_cells", "mts_compute_pair_forces",
           "mts_compute_triplet_forces", "mts_respa_step", "mts_sync", "mts_last_error",
           "mts_status_string", "mts_get_grid", "mts_get_cell_index", "mts_count_triplets",
           "mts_list_triplets", "mts_enable_kernel_timing", "mts_kernel_times", "mts_set_option",
           "mts_autotune", "mts_get_tuning", "mts_compute_triplet_forces_static")
MTS_STATIC_SCRATCH_BYTES = 16 << 20
MTS_OPT_CYCLE_GRAPH = 1
MTS_OPT_LIST_LANES = 2
MTS_OPT_TILE_CLASSES = 3
MTS_OPT_F3_GATHER_APART = 4


class MTSError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        name = _status_name(code)
        super().__init__("%s failed: %s%s" % (what, name, (" (" + detail + ")") if detail else ""))
        self.code = code


class mts_params(C.Structure):
    _fields_ = [("epsilon", C.c_double), ("sigma", C.c_double), ("rc_pair", C.c_double),
                ("nu", C.c_double), ("rc_triplet", C.c_double), ("mass", C.c_double),
                ("dt", C.c_double), ("skin", C.c_double), ("k", C.c_int32),
                ("precision", C.c_int32),
                ("lj_energy_shift", C.c_int32), ("method", C.c_int32), ("k_outer", C.c_int32),
                ("rc_triplet_inner", C.c_double)]


class mts_tuning(C.Structure):
    _fields_ = [("skin", C.c_double), ("cell_factor", C.c_double), ("list_lanes", C.c_int32),
                ("stage_cap", C.c_int32), ("list_cap", C.c_int32), ("pair_cap", C.c_int32),
                ("nl_cap", C.c_int32), ("trials", C.c_int32), ("shared_launch", C.c_int32),
                ("tile_classes", C.c_int32), ("cycle_ms", C.c_double),
                ("tight_caps", C.c_int32), ("triplet_workgroups_per_cu", C.c_int32),
                ("f3_gather_apart", C.c_int32), ("pad_", C.c_int32)]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Loads libmts.so and declares its signatures.  Raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError("libmts.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2507_11172_amd/build.py" % path)
    # PyTorch ships its own HIP runtime under the same soname as the system one.  Loading
    # torch first makes libmts.so bind to that runtime, so that device pointers from torch
    # tensors and the library's own allocations live in one HIP context.
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp = C.c_void_p
    L.mts_init_system.argtypes = [C.POINTER(mts_params), C.c_int32, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double), vp, C.POINTER(vp)]
    L.mts_destroy_system.argtypes = [vp]
    L.mts_destroy_system.restype = None
    L.mts_build_cells.argtypes = [vp, vp]
    L.mts_compute_pair_forces.argtypes = [vp, vp, vp, vp]
    L.mts_compute_triplet_forces.argtypes = [vp, vp, vp, vp]
    L.mts_respa_step.argtypes = [vp, vp, vp, C.c_int64, vp]
    L.mts_sync.argtypes = [vp]
    L.mts_last_error.argtypes = [vp]
    L.mts_last_error.restype = C.c_char_p
    L.mts_status_string.argtypes = [C.c_int32]
    L.mts_status_string.restype = C.c_char_p
    L.mts_get_grid.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    L.mts_get_cell_index.argtypes = [vp, vp]
    L.mts_count_triplets.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    L.mts_list_triplets.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    L.mts_enable_kernel_timing.argtypes = [vp, C.c_int32]
    L.mts_set_option.argtypes = [vp, C.c_int32, C.c_int64]
    L.mts_set_option.restype = C.c_int32
    L.mts_kernel_times.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.mts_autotune.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(mts_tuning)]
    L.mts_get_tuning.argtypes = [vp, C.POINTER(mts_tuning)]
    L.mts_compute_triplet_forces_static.argtypes = [C.POINTER(mts_params), C.c_int64,
                                                    C.POINTER(C.c_double), vp, vp, vp, vp]
    for name in ("mts_enable_kernel_timing", "mts_kernel_times", "mts_init_system",
                 "mts_build_cells", "mts_compute_pair_forces", "mts_compute_triplet_forces",
                 "mts_respa_step", "mts_sync", "mts_get_grid", "mts_get_cell_index",
                 "mts_count_triplets", "mts_list_triplets", "mts_autotune", "mts_get_tuning",
                 "mts_compute_triplet_forces_static"):
        getattr(L, name).restype = C.c_int32
    _LIB = L
    return L


def _status_name(code: int) -> str:
    try:
        return load_library().mts_status_string(code).decode()
    except Exception:
        return "status %d" % code


@dataclass
class Params:
    epsilon: float = 1.0
    sigma: float = 1.0
    rc_pair: float = 2.5
    nu: float = 0.073
    rc_triplet: float = 2.5
    mass: float = 1.0
    dt: float = 0.001
    k: int = 1
    precision: str = "fp64"   # "fp64" or "fp32"
    lj_energy_shift: bool = True
    skin: float = 0.0         # pair-list skin; 0 picks the library default
    method: str = "cutoff"    # "cutoff" (linked cells, periodic) or "direct" (DirectSum)
    k_outer: int = 1          # > 1: nested r-RESPA, outer triplet class every k * k_outer steps
    rc_triplet_inner: float = 0.0  # split of the two triplet distance classes (k_outer > 1)

    @classmethod
    def algorithm1(cls, delta_t: float, P: int, **kw) -> "Params":
        """Parameters running Algorithm 1 (Sec. 2.3.1): full steps delta_t of P sub-steps,
        F2 in the sub-steps and F3 kicks per full step -- the same scheme as Algorithm 2
        with dt = delta_t / P and step-size factor P."""
        if P < 1:
            raise ValueError("P must be >= 1")
        return cls(dt=delta_t / P, k=int(P), **kw)

    @property
    def span(self) -> int:
        """Inner steps per full step (k, times k_outer when nested)."""
        return self.k * max(1, self.k_outer)

    def to_c(self) -> mts_params:
        prec = {"fp64": MTS_FP64, "fp32": MTS_FP32}[self.precision]
        meth = {"cutoff": MTS_CUTOFF, "direct": MTS_DIRECT}[self.method]
        return mts_params(self.epsilon, self.sigma, self.rc_pair, self.nu, self.rc_triplet,
                          self.mass, self.dt, float(self.skin), int(self.k), prec,
                          int(bool(self.lj_energy_shift)), meth, int(self.k_outer),
                          float(self.rc_triplet_inner))


def _ptr(t, what: str, shape: Optional[Tuple[int, ...]] = None, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % what)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (what, shape, tuple(t.shape)))
    return C.c_void_p(t.data_ptr())


def compute_triplet_forces_static(params: Params, box, x, f3, ew=None, stream=None):
    """mts_compute_triplet_forces_static: F3 (and {U3, W3} into ew) of one periodic system
    without a handle and without device allocation (synchronising)."""
    import numpy as np
    import torch
    lib = load_library()
    n = int(x.shape[0]) if x is not None else 0
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
    if stream is None:
        stream = torch.cuda.current_stream()
    cp = params.to_c()
    rc = lib.mts_compute_triplet_forces_static(
        C.byref(cp), n, b.ctypes.data_as(C.POINTER(C.c_double)),
        _ptr(x, "x", (n, 3), torch.float64), _ptr(f3, "f3", (n, 3), torch.float64),
        _ptr(ew, "ew", (2,), torch.float64), C.c_void_p(stream.cuda_stream))
    if rc != MTS_OK:
        raise MTSError(rc, "mts_compute_triplet_forces_static")


class System:
    """One mts_system handle: n_systems periodic boxes, concatenated particles."""

    def __init__(self, params: Params, n_particles: Sequence[int], box, stream=None):
        import numpy as np
        import torch
        self._lib = load_library()
        self.params = params
        self.n_particles = [int(v) for v in n_particles]
        self.n_systems = len(self.n_particles)
        self.n = sum(self.n_particles)
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(self.n_systems, 3))
        np_ = np.ascontiguousarray(np.asarray(self.n_particles, dtype=np.int64))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = C.c_void_p()
        cp = params.to_c()
        rc = self._lib.mts_init_system(C.byref(cp), self.n_systems,
                                       np_.ctypes.data_as(C.POINTER(C.c_int64)),
                                       b.ctypes.data_as(C.POINTER(C.c_double)),
                                       C.c_void_p(stream.cuda_stream), C.byref(handle))
        if rc != MTS_OK:
            raise MTSError(rc, "mts_init_system")
        self._h = handle

    # -- helpers
    def _check(self, rc: int, what: str):
        if rc != MTS_OK:
            detail = self._lib.mts_last_error(self._h).decode()
            raise MTSError(rc, what, detail)

    def _vec(self, t, what):
        import torch
        return _ptr(t, what, (self.n, 3), torch.float64)

    # -- C ABI mirror
    def build_cells(self, x):
        self._check(self._lib.mts_build_cells(self._h, self._vec(x, "x")), "mts_build_cells")

    def compute_pair_forces(self, x, f2, ew=None):
        import torch
        self._check(self._lib.mts_compute_pair_forces(
            self._h, self._vec(x, "x"), self._vec(f2, "f2"),
            _ptr(ew, "ew", (self.n_systems, 2), torch.float64)), "mts_compute_pair_forces")

    def compute_triplet_forces(self, x, f3, ew=None):
        import torch
        self._check(self._lib.mts_compute_triplet_forces(
            self._h, self._vec(x, "x"), self._vec(f3, "f3"),
            _ptr(ew, "ew", (self.n_systems, 2), torch.float64)), "mts_compute_triplet_forces")

    def respa_step(self, x, v, n_iter: int, e_full=None):
        import torch
        span = self.params.span
        shape = (n_iter // span + 1, self.n_systems, MTS_NE) if span > 0 else None
        self._check(self._lib.mts_respa_step(
            self._h, self._vec(x, "x"), self._vec(v, "v"), int(n_iter),
            _ptr(e_full, "e_full", shape, torch.float64)), "mts_respa_step")

    def sync(self):
        self._check(self._lib.mts_sync(self._h), "mts_sync")

    def get_grid(self, system: int = 0) -> Tuple[int, int, int]:
        out = (C.c_int32 * 3)()
        self._check(self._lib.mts_get_grid(self._h, int(system), out), "mts_get_grid")
        return tuple(int(v) for v in out)

    def get_cell_index(self, out):
        import torch
        self._check(self._lib.mts_get_cell_index(self._h, _ptr(out, "cell", (self.n,), torch.int32)),
                    "mts_get_cell_index")

    def count_triplets(self, x) -> int:
        c = C.c_int64(0)
        self._check(self._lib.mts_count_triplets(self._h, self._vec(x, "x"), C.byref(c)),
                    "mts_count_triplets")
        return int(c.value)

    def list_triplets(self, x, cap: int):
        """(ijk [M, 3] int32 device tensor, total count)."""
        import torch
        buf = torch.zeros((max(cap, 1), 3), dtype=torch.int32, device=x.device)
        c = C.c_int64(0)
        self._check(self._lib.mts_list_triplets(self._h, self._vec(x, "x"), _ptr(buf, "ijk"),
                                                int(cap), C.byref(c)), "mts_list_triplets")
        total = int(c.value)
        return buf[:min(total, cap)], total

    @staticmethod
    def _tuning_dict(t: "mts_tuning") -> dict:
        return {name: getattr(t, name) for name, _ in mts_tuning._fields_ if name != "pad_"}

    def autotune(self, x, v, budget_ms: int = 2000) -> dict:
        """Times candidate configurations on (x, v) (not modified) and keeps the fastest;
        returns it as a dict (see mts_tuning)."""
        t = mts_tuning()
        self._check(self._lib.mts_autotune(self._h, self._vec(x, "x"), self._vec(v, "v"),
                                           int(budget_ms), C.byref(t)), "mts_autotune")
        return self._tuning_dict(t)

    def tuning(self) -> dict:
        t = mts_tuning()
        self._check(self._lib.mts_get_tuning(self._h, C.byref(t)), "mts_get_tuning")
        return self._tuning_dict(t)

    def set_option(self, option: int, value: int):
        self._check(self._lib.mts_set_option(self._h, int(option), int(value)), "mts_set_option")

    def enable_kernel_timing(self, enable: bool = True):
        self._check(self._lib.mts_enable_kernel_timing(self._h, int(bool(enable))),
                    "mts_enable_kernel_timing")

    def kernel_times(self):
        """{"triplet": (launches, ms), "pair": (launches, ms)} since the last call."""
        n = (C.c_int64 * 2)()
        ms = (C.c_double * 2)()
        self._check(self._lib.mts_kernel_times(self._h, n, ms), "mts_kernel_times")
        return {"triplet": (int(n[0]), float(ms[0])), "pair": (int(n[1]), float(ms[1]))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mts_destroy_system(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
