// Linked-cell binning by counting sort (Sec. 2.2 and 4.1: particles are assigned to
// cells by position).  Steps: wrap + cell index + histogram (int atomics), exclusive
// scan (which also clears the histogram for the next call), atomic scatter, then a rank
// pass that restores ascending input order inside every cell -- the sort is stable and
// deterministic, which fixes every later summation order.  All passes are HBM/L2-bound
// streaming kernels.  One launch per pass serves both cell grids (blockIdx.y selects
// the grid), so a rebinning of the pair-list and triplet grids costs four launches.
#include <algorithm>

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
    // Arrival slot inside the cell, one device atomic per distinct cell of the wavefront
    // (particles in input order are mostly clustered in space, and these atomics are
    // resolved far from the CU): group the lanes by cell, the lowest lane of each group
    // adds the group's size, the others take consecutive slots after it.  Any unique slot
    // will do -- the rank pass orders every cell by input index.
    uint64_t todo = __builtin_amdgcn_read_exec(), group = 0;
    while (todo) {
        const int l = __builtin_ctzll(todo);
        const int lc = __builtin_amdgcn_readlane(cell, l);
        const uint64_t m = ballot(cell == lc) & todo;
        if (cell == lc) group = m;
        todo &= ~m;
    }
    const int leader = __builtin_ctzll(group);
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    int base = 0;
    if (lane == leader) base = atomicAdd(&g.count[cell], __popcll(group));
    base = __shfl(base, leader);
    g.rank[i] = base + (int)__builtin_amdgcn_mbcnt_hi(
                           (unsigned)(group >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)group, 0u));
}

// Exclusive scan of count[0..ncell) into start[0..ncell], start[ncell] = n, over many
// workgroups that never wait for one another:
//  * k_scan_tiles: one workgroup of 1024 threads per tile of kScanTile cells (each thread
//    four consecutive counts) writes the tile-local exclusive prefix to start_loc and the
//    tile total to tile_sum, and clears the counts for the next binning.  The workgroup
//    that finishes last (a device-scope counter, reset by it) scans the tile totals into
//    tile_off and writes start[ncell].
//  * k_bin_scatter adds the tile offsets back: start = start_loc + tile_off[tile], both
//    for its own scatter and, grid-stride, into start[] for every later kernel.
// Integer sums: the result does not depend on the order.
__global__ void __launch_bounds__(1024) k_scan_tiles(BinArgs a) {
    constexpr int kWaves = 1024 / kWave;
    __shared__ int wsum[kWaves];
    __shared__ bool last;
    const BinGrid &g = a.g[blockIdx.y];
    const int ncell = g.ncell;
    const int ntile = (ncell + kScanTile - 1) / kScanTile;
    const int tile = blockIdx.x;
    if (tile >= ntile) return;  // grids of fewer tiles (uniform per workgroup)
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int c0 = tile * kScanTile + 4 * t;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = c0 + k < ncell ? g.count[c0 + k] : 0;
    const int s = (v[0] + v[1]) + (v[2] + v[3]);
    // inclusive scan across the lanes of each wavefront, then of the wavefront totals
    int incl = s;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const int y = __shfl_up(incl, m);
        if (lane >= m) incl += y;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const int w = lane < kWaves ? wsum[lane] : 0;
        int wi = w;
#pragma unroll
        for (int m = 1; m < kWaves; m <<= 1) {
            const int y = __shfl_up(wi, m);
            if (lane >= m) wi += y;
        }
        if (lane < kWaves) wsum[lane] = wi - w;  // exclusive prefix of each wavefront
    }
    __syncthreads();
    int run = wsum[wave] + incl - s;  // exclusive prefix of this thread's four cells in the tile
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (c0 + k < ncell) {
            g.start_loc[c0 + k] = run;
            run += v[k];
            g.count[c0 + k] = 0;
        }
    if (t == 1023) g.tile_sum[tile] = wsum[kWaves - 1] + incl;
    __threadfence();
    __syncthreads();
    if (t == 0) last = atomicAdd(&g.tile_sum[2 * ntile], 1) == ntile - 1;
    __syncthreads();
    if (!last) return;
    // the last tile: exclusive scan of the ntile totals (a few dozen) by thread 0
    __threadfence();
    if (t == 0) {
        int acc = 0;
        for (int q = 0; q < ntile; ++q) {
            const int x = __hip_atomic_load(&g.tile_sum[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            g.tile_sum[ntile + q] = acc;
            acc += x;
        }
        g.start[ncell] = (int)a.n;
        g.tile_sum[2 * ntile] = 0;  // counter at rest for the next binning
    }
}

// Scatter of every particle to its cell (arrival rank inside the cell), and the final
// cell starts: start = start_loc + the offset of the cell's tile.
__global__ void __launch_bounds__(256) k_bin_scatter(BinArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const BinGrid &g = a.g[blockIdx.y];
    const int *off = g.tile_sum + (g.ncell + kScanTile - 1) / kScanTile;
    if (i < a.n) {
        const int c = g.cell_of[i];
        g.tmp[g.start_loc[c] + off[c / kScanTile] + g.rank[i]] = (int)i;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = i; c < g.ncell; c += stride) g.start[c] = g.start_loc[c] + off[c / kScanTile];
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
    if (g.x_ref) {  // in the grid's sorted order, like xs
        g.x_ref[3 * dst] = w.x;
        g.x_ref[3 * dst + 1] = w.y;
        g.x_ref[3 * dst + 2] = w.z;
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
    int ntile = 0;
    for (int q = 0; q < a.ng; ++q) {
        if (a.g[q].ncell <= 0) return hipErrorInvalidValue;
        ntile = std::max(ntile, (a.g[q].ncell + kScanTile - 1) / kScanTile);
    }
    if (a.n > 0) k_bin_count<<<grid, 256, 0, st>>>(a);
    k_scan_tiles<<<dim3((unsigned)ntile, (unsigned)a.ng), 1024, 0, st>>>(a);
    // also for n = 0: the scatter writes the final cell starts
    k_bin_scatter<<<dim3(std::max(1u, grid.x), (unsigned)a.ng), 256, 0, st>>>(a);
    if (a.n > 0) k_rank_gather<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_local_cell_index(hipStream_t st, int64_t n, const int *cell_of,
                                   const SysDesc *sd, const int *sys_of, int *out) {
    if (n > 0) k_local_cell_index<<<blocks_for(n, 256), 256, 0, st>>>(n, cell_of, sd, sys_of, out);
    return hipGetLastError();
}

}  // namespace mts
