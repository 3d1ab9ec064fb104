// Linked-cell binning by counting sort (Sec. 2.2 and 4.1: particles are assigned to
// cells by position).  Steps: wrap + cell index + histogram (int atomics), exclusive
// scan (which also clears the histogram for the next call), atomic scatter, then a rank
// pass that restores ascending input order inside every cell -- the sort is stable and
// deterministic, which fixes every later summation order.  All passes are HBM/L2-bound
// streaming kernels.  One launch per pass serves both cell grids (blockIdx.y selects
// the grid), so a rebinning of the pair-list and triplet grids costs four launches.
#include "common.h"

namespace mts {

__global__ void __launch_bounds__(256) k_bin_count(BinArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const BinGrid &g = a.g[blockIdx.y];
    const SysDesc &d = g.sd[a.sys_of[i]];
    int c[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double xi = a.x[3 * i + k];
        finite = finite && isfinite(xi);
        c[k] = cell_coord(wrap1(xi, d.L[k]), d.q[k], d.nc[k]);
    }
    if (!finite) atomicOr(a.flags, kFlagNonFinite);
    const int cell = d.cell0 + (c[2] * d.nc[1] + c[1]) * d.nc[0] + c[0];
    g.cell_of[i] = cell;
    g.rank[i] = atomicAdd(&g.count[cell], 1);
}

// Exclusive scan of count[0..ncell) into start[0..ncell], start[ncell] = n.  One
// workgroup of 1024 threads per grid walks the cells in tiles of 4,096: each thread loads
// four consecutive counts (consecutive threads, consecutive 16-byte runs), the workgroup
// scans the 1,024 thread sums in LDS, and a running carry links the tiles.  The counts
// are cleared for the next binning.  Integer sums: the result does not depend on the order.
__global__ void __launch_bounds__(1024) k_scan(BinArgs a) {
    __shared__ int part[1024];
    const BinGrid &g = a.g[blockIdx.x];
    const int ncell = g.ncell;
    const int t = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < ncell; base += 4 * 1024) {
        const int c0 = base + 4 * t;
        int v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = c0 + k < ncell ? g.count[c0 + k] : 0;
        const int s = (v[0] + v[1]) + (v[2] + v[3]);
        part[t] = s;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int u = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        int run = carry + part[t] - s;  // exclusive prefix of this thread's four cells
        carry += part[1023];
        __syncthreads();  // every thread has read part[] before the next tile writes it
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncell) {
                g.start[c0 + k] = run;
                run += v[k];
                g.count[c0 + k] = 0;
            }
    }
    if (t == 0) g.start[ncell] = (int)a.n;
}

__global__ void __launch_bounds__(256) k_bin_scatter(BinArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const BinGrid &g = a.g[blockIdx.y];
    g.tmp[g.start[g.cell_of[i]] + g.rank[i]] = (int)i;
}

// Final, deterministic order inside each cell: the particle that the atomic scatter put
// at slot p finds its rank among the cell's members by counting smaller input indices
// (cells hold ~10-30 particles), then writes its input index and its wrapped position
// to the ranked slot.  Equal cells therefore keep ascending input order.
__global__ void __launch_bounds__(256) k_rank_gather(BinArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const BinGrid &g = a.g[blockIdx.y];
    const int key = g.tmp[p];
    const int c = g.cell_of[key];
    const int b = g.start[c], e = g.start[c + 1];
    int r = 0;
    for (int q = b; q < e; ++q) r += g.tmp[q] < key;
    const int64_t dst = b + r;
    g.perm[dst] = key;
    g.inv_perm[key] = (int)dst;
    const SysDesc &d = g.sd[a.sys_of[key]];
    Pos4 w;
    w.x = wrap1(a.x[3 * (int64_t)key], d.L[0]);
    w.y = wrap1(a.x[3 * (int64_t)key + 1], d.L[1]);
    w.z = wrap1(a.x[3 * (int64_t)key + 2], d.L[2]);
    w.w = 0.0;
    g.xs[dst] = w;
    if (g.x_ref) {
        g.x_ref[3 * (int64_t)key] = w.x;
        g.x_ref[3 * (int64_t)key + 1] = w.y;
        g.x_ref[3 * (int64_t)key + 2] = w.z;
    }
}

__global__ void k_local_cell_index(int64_t n, const int *__restrict__ cell_of,
                                   const SysDesc *__restrict__ sd, const int *__restrict__ sys_of,
                                   int *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = cell_of[i] - sd[sys_of[i]].cell0;
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_bin(hipStream_t st, const BinArgs &a) {
    if (a.ng < 1 || a.ng > 2) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(a.n, 256), (unsigned)a.ng);
    if (a.n > 0 && !a.counted) k_bin_count<<<grid, 256, 0, st>>>(a);
    k_scan<<<(unsigned)a.ng, 1024, 0, st>>>(a);  // also for n = 0: start[] must be valid
    if (a.n > 0) {
        k_bin_scatter<<<grid, 256, 0, st>>>(a);
        k_rank_gather<<<grid, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_local_cell_index(hipStream_t st, int64_t n, const int *cell_of,
                                   const SysDesc *sd, const int *sys_of, int *out) {
    if (n > 0) k_local_cell_index<<<blocks_for(n, 256), 256, 0, st>>>(n, cell_of, sd, sys_of, out);
    return hipGetLastError();
}

}  // namespace mts
