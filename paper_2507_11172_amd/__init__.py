"""MI355X-native two- plus three-body molecular dynamics with r-RESPA.

The compute path is libmts.so (HIP kernels for gfx950 behind the C ABI of
include/mts.h); ``paper_2507_11172_amd.mts`` is its ctypes binding and
``paper_2507_11172_amd.workloads`` builds seeded synthetic inputs.
"""
__all__ = ["mts", "workloads"]
