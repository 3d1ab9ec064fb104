// Linked-cell binning by counting sort (Sec. 2.2 and 4.1: particles are assigned to
// cells by position).  Steps: wrap + cell index + histogram (int atomics), exclusive
// scan (which also clears the histogram for the next call), atomic scatter, then a rank
// pass that restores ascending input order inside every cell -- the sort is stable and
// deterministic, which fixes every later summation order.  All passes are HBM/L2-bound
// streaming kernels.
#include "common.h"

namespace mts {

__global__ void __launch_bounds__(256) k_bin_count(int64_t n, const double *__restrict__ x,
                                                   const SysDesc *__restrict__ sd,
                                                   const int *__restrict__ sys_of,
                                                   int *__restrict__ cell_of,
                                                   int *__restrict__ rank, int *count,
                                                   int *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const SysDesc &d = sd[sys_of[i]];
    int c[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double xi = x[3 * i + k];
        finite = finite && isfinite(xi);
        c[k] = cell_coord(wrap1(xi, d.L[k]), d.q[k], d.nc[k]);
    }
    if (!finite) atomicOr(flags, kFlagNonFinite);
    int cell = d.cell0 + (c[2] * d.nc[1] + c[1]) * d.nc[0] + c[0];
    cell_of[i] = cell;
    rank[i] = atomicAdd(&count[cell], 1);
}

// Exclusive scan of count[0..ncell) into start[0..ncell], start[ncell] = n_total.
// One workgroup of 1024 threads; each thread owns a contiguous chunk.
__global__ void __launch_bounds__(1024) k_scan(int ncell, int *__restrict__ count,
                                               int *__restrict__ start, int64_t n_total) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int chunk = (ncell + 1023) / 1024;
    const int b = t * chunk;
    const int e = min(ncell, b + chunk);
    int s = 0;
    for (int c = b; c < e; ++c) s += count[c];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;  // exclusive prefix of this chunk
    for (int c = b; c < e; ++c) {
        start[c] = run;
        run += count[c];
        count[c] = 0;  // ready for the next binning
    }
    if (t == 0) start[ncell] = (int)n_total;
}

__global__ void __launch_bounds__(256) k_bin_scatter(int64_t n, const int *__restrict__ cell_of,
                                                     const int *__restrict__ rank,
                                                     const int *__restrict__ start,
                                                     int *__restrict__ perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[start[cell_of[i]] + rank[i]] = (int)i;
}

// Final, deterministic order inside each cell: the particle that the atomic scatter put
// at slot p finds its rank among the cell's members by counting smaller input indices
// (cells hold ~10-20 particles), then writes its input index and its wrapped position
// (SoA) to the ranked slot.  Equal cells therefore keep ascending input order.
__global__ void __launch_bounds__(256) k_rank_gather(int64_t n, const int *__restrict__ tmp,
                                                     const int *__restrict__ cell_of,
                                                     const int *__restrict__ start,
                                                     const double *__restrict__ x,
                                                     const SysDesc *__restrict__ sd,
                                                     const int *__restrict__ sys_of,
                                                     int *__restrict__ perm,
                                                     int *__restrict__ inv_perm,
                                                     double *__restrict__ xs,
                                                     double *__restrict__ x_ref) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int key = tmp[p];
    const int c = cell_of[key];
    const int b = start[c], e = start[c + 1];
    int r = 0;
    for (int q = b; q < e; ++q) r += tmp[q] < key;
    const int64_t dst = b + r;
    perm[dst] = key;
    inv_perm[key] = (int)dst;
    const SysDesc &d = sd[sys_of[key]];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double w = wrap1(x[3 * (int64_t)key + k], d.L[k]);
        xs[k * n + dst] = w;
        if (x_ref) x_ref[3 * (int64_t)key + k] = w;
    }
}

__global__ void k_local_cell_index(int64_t n, const int *__restrict__ cell_of,
                                   const SysDesc *__restrict__ sd, const int *__restrict__ sys_of,
                                   int *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = cell_of[i] - sd[sys_of[i]].cell0;
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_bin_count(hipStream_t st, int64_t n, const double *x, const SysDesc *sd,
                            const int *sys_of, int *cell_of, int *rank, int *count, int *flags) {
    if (n > 0)
        k_bin_count<<<blocks_for(n, 256), 256, 0, st>>>(n, x, sd, sys_of, cell_of, rank, count, flags);
    return hipGetLastError();
}

hipError_t launch_scan(hipStream_t st, int ncell, int *count, int *start, int64_t n_total) {
    k_scan<<<1, 1024, 0, st>>>(ncell, count, start, n_total);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(hipStream_t st, int64_t n, const int *cell_of, const int *rank,
                              const int *start, int *perm) {
    if (n > 0) k_bin_scatter<<<blocks_for(n, 256), 256, 0, st>>>(n, cell_of, rank, start, perm);
    return hipGetLastError();
}

hipError_t launch_rank_gather(hipStream_t st, int64_t n, const int *tmp, const int *cell_of,
                              const int *start, const double *x, const SysDesc *sd,
                              const int *sys_of, int *perm, int *inv_perm, double *xs,
                              double *x_ref) {
    if (n > 0)
        k_rank_gather<<<blocks_for(n, 256), 256, 0, st>>>(n, tmp, cell_of, start, x, sd, sys_of,
                                                          perm, inv_perm, xs, x_ref);
    return hipGetLastError();
}

hipError_t launch_local_cell_index(hipStream_t st, int64_t n, const int *cell_of,
                                   const SysDesc *sd, const int *sys_of, int *out) {
    if (n > 0) k_local_cell_index<<<blocks_for(n, 256), 256, 0, st>>>(n, cell_of, sd, sys_of, out);
    return hipGetLastError();
}

}  // namespace mts
