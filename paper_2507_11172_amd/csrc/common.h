// Internal declarations of the MI355X r-RESPA library: device system descriptors,
// canonical periodic geometry, stencil tables and the kernel launchers.
//
// Every source of the library is compiled with -ffp-contract=off: the cutoff
// geometry (wrap, minimum image, squared distance) must round exactly as written, so
// that cell assignment and the interacting pair/triplet sets are reproducible
// bit for bit.  Force arithmetic that wants fused multiply-adds spells them out
// with fma()/fmaf().
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mts {

constexpr int kWave = 64;        // CDNA wavefront width

// Lanes of the wavefront where p holds, as a 64-bit mask.  Taken from the bool itself, so
// the compare's lane mask is used directly (through an int, the predicate would first be
// materialised in a vector register and compared again).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
constexpr int kNumHalf = 14;     // self cell + 13 forward cells of the half stencil
constexpr int kNumFull = 27;     // full 3x3x3 stencil
constexpr int kNE = 5;           // K, U2, U3, W2, W3

// Per-system description, read by every kernel.
struct SysDesc {
    double L[3];    // box edges
    double q[3];    // n_cells / L, the cell-coordinate scale
    double iL[3];   // 1 / L
    int nc[3];      // cells per edge (>= 2); cell edge L/nc exceeds the largest cutoff
    int cell0;      // first global cell id of this system
    int ncell;      // nc[0] * nc[1] * nc[2]
    int whole;      // triplet grid only, 1 when ncell < 14: the half stencil would stage
                    // particles of the system more than once, so the triplet kernel stages
                    // the whole system instead, and cell c stands for anchor chunk c
    int64_t p0;     // first particle (global index); particles are concatenated by system
    int64_t n;      // particles in this system
};

// Sorted wrapped position, padded to 32 bytes so that a gather of one particle touches
// a single cache line and a staged copy is two 16-byte loads.
struct alignas(32) Pos4 {
    double x, y, z, w;  // w = 0
};

// Device error flags (bit mask in a single int).
enum : int {
    kFlagStageOverflow = 1,  // a triplet neighbourhood did not fit the LDS tile
    kFlagListOverflow = 2,   // an anchor had more forward neighbours than the list holds
    kFlagNonFinite = 4,      // a force or energy was NaN/Inf
    kFlagTripletListFull = 8,// debug triplet listing exceeded its buffer (not an error)
    kFlagSkin = 16,          // a particle moved more than half the pair-list skin
    kFlagPairList = 32       // a particle had more pair-list neighbours than the list holds
};

// ---------------------------------------------------------------- geometry
// Wrap into [0, L]: w = x - L * floor(x / L).  (w may equal L after rounding; the cell
// coordinate is clamped, so such a particle sits on the top face of the last cell.)
__device__ __forceinline__ double wrap1(double x, double L) { return x - L * floor(x / L); }

// Cell coordinate min(nc - 1, max(0, floor(w * q))); NaN maps to 0 (the bin kernel flags
// non-finite positions separately).
__device__ __forceinline__ int cell_coord(double w, double q, int nc) {
    const double t = floor(w * q);
    if (!(t >= 0.0)) return 0;
    return t < (double)nc ? (int)t : nc - 1;
}

// Cell coordinate c + o on a periodic grid of nc cells, and the image shift (in box
// edges: -1, 0, +1) that the particles of that cell carry when seen from cell c.
// Requires |o| <= 1 and nc >= 2.
__device__ __forceinline__ int wrap_cell(int c, int o, int nc, int &shift) {
    int t = c + o;
    shift = 0;
    if (t < 0) { t += nc; shift = -1; }
    else if (t >= nc) { t -= nc; shift = 1; }
    return t;
}

// Minimum-image displacement component from p to q.  The caller supplies the image
// shift S (0 or +-L) of q relative to p; the rounding is fl(fl(x_q - x_p) + S), which
// equals fl(d - L*rint(d/L)) for every pair within a cutoff below L/2.
__device__ __forceinline__ double disp1(double xp, double xq, double S) { return (xq - xp) + S; }

__device__ __forceinline__ double norm2(double dx, double dy, double dz) {
    return (dx * dx + dy * dy) + dz * dz;
}

// Offsets of the 3x3x3 stencil, full (index 13 is the centre) and forward half (index 0
// is the centre).  "Forward" is lexicographic in (z, y, x): oz > 0, or oz == 0 and
// oy > 0, or oz == oy == 0 and ox > 0.
__device__ __forceinline__ void full_offset(int o, int &ox, int &oy, int &oz) {
    ox = o % 3 - 1;
    oy = (o / 3) % 3 - 1;
    oz = o / 9 - 1;
}

__device__ __forceinline__ void half_offset(int o, int &ox, int &oy, int &oz) {
    // o = 0 is (0,0,0); o = 1..13 are full-stencil entries 14..26 (all forward).
    int f = o == 0 ? 13 : 13 + o;
    full_offset(f, ox, oy, oz);
}

// ---------------------------------------------------------------- tile staging
// Stencil description of one workgroup's tile: for each stencil cell o (< NC), the
// first sorted particle, the tile offset and the packed image-shift code.
template <int NC>
struct StencilTable {
    int begin[NC];
    int off[NC + 1];
    int code[NC];
};

// Fills the table for base cell (cx, cy, cz).  Lane o of wave 0 handles stencil cell o
// (offsets from `offset_of(o)`), reads its bounds from `start`, and a shuffle prefix sum
// gives the tile offsets, so a tile costs two dependent global loads instead of two per
// cell.  Call from every thread; contains __syncthreads().  Returns the total count.
template <int NC, bool HALF>
__device__ __forceinline__ int stencil_table(StencilTable<NC> &tab, const SysDesc &d, int cx,
                                             int cy, int cz, const int *start) {
    static_assert(NC <= 64, "one lane per stencil cell");
    const int tid = threadIdx.x;
    if (tid < 64) {
        int cnt = 0;
        if (tid < NC) {
            int ox, oy, oz, sx, sy, sz;
            if (HALF) {
                const int f = tid == 0 ? 13 : 13 + tid;
                ox = f % 3 - 1; oy = (f / 3) % 3 - 1; oz = f / 9 - 1;
            } else {
                ox = tid % 3 - 1; oy = (tid / 3) % 3 - 1; oz = tid / 9 - 1;
            }
            const int tx = wrap_cell(cx, ox, d.nc[0], sx);
            const int ty = wrap_cell(cy, oy, d.nc[1], sy);
            const int tz = wrap_cell(cz, oz, d.nc[2], sz);
            const int cell = d.cell0 + (tz * d.nc[1] + ty) * d.nc[0] + tx;
            const int b = start[cell];
            cnt = start[cell + 1] - b;
            tab.begin[tid] = b;
            tab.code[tid] = (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4) | (tid << 8);
        }
        int incl = cnt;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const int y = __shfl_up(incl, m);
            if (tid >= m) incl += y;
        }
        if (tid < NC) tab.off[tid] = incl - cnt;
        if (tid == NC - 1) tab.off[NC] = incl;
    }
    __syncthreads();
    return tab.off[NC];
}

// Stencil cell of tile entry t (binary search over the offsets).
template <int NC>
__device__ __forceinline__ int stencil_cell_of(const StencilTable<NC> &tab, int t) {
    int lo = 0, hi = NC - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab.off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().

// Cells per tile of the multi-workgroup scan.
constexpr int kScanTile = 4096;

// Binning (counting sort by cell) of one set of positions into one or two cell grids
// (the pair-list grid and the triplet grid) with one launch per pass.
struct BinGrid {
    const SysDesc *sd;
    int ncell;
    int *cell_of;           // [n] global cell id, input order
    int *rank;              // [n] arrival rank inside the cell (scratch)
    int *count;             // [ncell] histogram; zero on entry, left zero by the scan
    int *start;             // [ncell + 1] first sorted slot of each cell
    int *start_loc;         // [ncell] exclusive prefix of the counts inside each scan tile
    int *tile_sum;          // [2 ntile + 1], ntile = ceil(ncell / kScanTile): tile totals,
                            // tile offsets, and the scan's completion counter (zero at rest)
    int *tmp;               // [n] unordered scatter (scratch)
    int *perm;              // [n] sorted -> input index
    int *inv_perm;          // [n] input -> sorted index
    Pos4 *xs;               // [n] sorted wrapped positions
    double *x_ref;          // [n][3] wrapped positions in this grid's sorted order, or null
};
struct BinArgs {
    int64_t n;
    const double *x;        // [n][3] positions, any image
    const int *sys_of;      // [n]
    int *flags;
    int ng;                 // 1 or 2 grids
    BinGrid g[2];
};
hipError_t launch_bin(hipStream_t st, const BinArgs &a);
// Local (per-system) cell index of every particle, input order.
hipError_t launch_local_cell_index(hipStream_t st, int64_t n, const int *cell_of,
                                   const SysDesc *sd, const int *sys_of, int *out);

struct PairArgs {
    int ncell;
    const int *sys_of_cell; // [ncell]
    int stage_cap;          // LDS tile capacity (particles)
    int64_t n;
    const Pos4 *xs;         // [n] sorted wrapped positions
    const int *perm;        // sorted -> input index
    const int *start;       // cell starts [ncell_total + 1]
    const SysDesc *sd;
    const int *sys_of;      // per particle (same in input and sorted order)
    double *f;              // out [n][3], input order (sorted with out_sorted)
    double *pe;             // out [n][2] per-particle {U2/2-sums, W2/2-sums}, sorted order
    double eps, sigma2, rc2, ushift;
    int *flags;
};
hipError_t launch_pair(hipStream_t st, const PairArgs &a);  // LJ in FP64 in both forms

// Verlet pair list of the pair grid: for every sorted particle p, the sorted indices of
// all particles within sqrt(rv2) (tile order), nbr[p * nl_cap + s], and their number
// nn[p].  The distance test runs in FP32 on positions relative to the base cell, with a
// relative margin that covers its rounding, so the list holds at least every pair
// within the list radius.
struct ListBuildArgs {
    int ncell;
    const int *sys_of_cell;
    int stage_cap;          // LDS tile capacity (particles)
    int64_t n;
    const Pos4 *xs;
    const int *start;
    const SysDesc *sd;
    int *nbr;
    int *nn;
    int nl_cap;
    double rv2;
    int *flags;
    int *stats;             // optional: [2] atomic max of the tile size and the row length
};
hipError_t launch_list_build(hipStream_t st, const ListBuildArgs &a);
size_t list_build_lds_bytes(int stage_cap);

// Pair forces from the pair list, fused with the r-RESPA update of each particle.  The
// displacement of each listed pair is re-derived from the current wrapped positions with
// the minimum image, so particles may wrap across the box between rebuilds.  After its
// force F = F2(x) is summed, particle p (input index q = perm[p]) is updated in
// Algorithm 2's order with the same expressions as k_int (see IntArgs), F taking the
// place of F2(x^i):
//   kick2:  v <- v + dt/(2m) (f2prev + F)
//   kick3:  v <- v + dt s/(2m) F3, for kick3_end and again for kick3_start
//   drift:  x <- wrap(x + dt v + dt^2/(2m) F), written to x (input order) and to xs_out
//           (sorted), and checked against x_ref (skin).
// xs (read) and xs_out (written) must be different buffers.
struct PairListArgs {
    int64_t n;
    const Pos4 *xs;         // current wrapped positions in the list's sorted order
    const int *perm;        // sorted -> input index
    int lanes;              // lanes per particle: 4, 8 or 16
    const int *nbr;         // [n][nl_cap]
    const int *nn;          // [n]
    int nl_cap;
    const SysDesc *sd;
    const int *sys_of;
    double *f;              // out [n][3], input order
    double *pe;             // out [n][2], sorted order, or null (no energies)
    double eps, sigma2, rc2, ushift;
    int *flags;
    // fused update (all optional)
    int kick2, kick3_end, kick3_start, drift;
    // The inner steps between the first and the last of a cycle keep v and F2 in the
    // pair grid's sorted order (coalesced): in_sorted reads v_in and f2prev at the sorted
    // index, out_sorted writes f and v_out there.  The drift takes x^i from xs (the same
    // bits as the input-order copy) and writes x (input order) only when x is non-null.
    int in_sorted, out_sorted;
    double *x;              // [n][3] input order, or null
    const double *v_in;     // [n][3]
    double *v_out;          // [n][3] (may be v_in)
    const double *f2prev;   // F2 of the previous inner position (kick2)
    const double *f3;       // F3 (kick3)
    double c2, c3, dt, cx;
    Pos4 *xs_out;           // [n] sorted positions after the drift
    // The next cycle's opening fused into a cycle's closing launch (optional): its F3 half
    // kick on the closed v and its first drift with this launch's F2, from x (input
    // order), into v_next, f2_next (sorted order) and xs_next, with the skin check; the
    // closed v, F2 and x stay as they are (the caller's output and the energy record)
    int open_next;
    double *v_next, *f2_next;
    Pos4 *xs_next;
    const double *x_ref;    // positions at the last list build (sorted order)
    double half_skin2;
    // optional: F3 gathered here from the triplet kernel's partial slots (fixed slot
    // order, as k_triplet_gather), written to f3_out and used by the kicks instead of f3
    const double *pf;       // [14][3][n] partial slots, or null
    const int *inv_perm3;   // input -> sorted index of the triplet grid
    double *f3_out;         // [n][3]
};
hipError_t launch_pair_list(hipStream_t st, const PairListArgs &a);  // LJ in FP64
size_t pair_lds_bytes(int stage_cap);

// Lets every LDS-tiled kernel use up to max_bytes of dynamic LDS per workgroup.
// LDS left to the kernels' static arrays when the dynamic limit is set (the triplet
// kernels' static LDS is at most 1.5 KB).
constexpr size_t kStaticLdsReserve = 2048;
hipError_t configure_kernel_lds(size_t max_bytes);

// Triplet forces: one launch whose workgroups take one base cell (item) each, in the order
// of cell_map, staging its forward half stencil (or a tiny system whole) in LDS; the
// pair-list build's cells follow as further items of the same launch.
struct TripletArgs {
    int ncell;              // base cells of this launch (items)
    const int *cell_map;    // [ncell] triplet-grid cell of each item, or nullptr: item b
                            // is cell b
    int any_whole;          // 1 if some system of the launch is staged whole (SysDesc.whole)
    int occ6;               // 1: six workgroups per CU fit this launch's LDS; its plain
                            // (unweighted) passes use the variants held to 80 VGPRs
    const Pos4 *xs;
    const int *start;
    const SysDesc *sd;
    const int *sys_of_cell; // [ncell]
    const int *perm;        // for triplet listing
    double *pf;             // out partial slots [kNumHalf][3][n]
    double *ce;             // out per-cell {U3, W3} [ncell][2]
    long long *cc;          // out per-cell triplet counts [ncell], or null
    int64_t n;
    double nu, rc2;
    int stage_cap, list_cap;
    int *flags;
    int *list_ijk;          // optional triplet listing [list_cap_rows][3]
    unsigned long long *list_n;  // listing counter
    long long list_rows;
    int *stats;             // optional: [2] atomic max of the tile size and of the anchor
                            // list length before capping
    int *tile_obs;          // [nsys] atomic max of the tile size per system, recorded on
                            // overflow and whenever stats is set
    // nested r-RESPA full step (w_out > 1): forces of triplets whose longest edge exceeds
    // sqrt(ra2) are scaled by w_out (energies and virials are not)
    double ra2, w_out;
};
hipError_t launch_triplet(hipStream_t st, const TripletArgs &a, bool fp32, bool listing);
// One launch: the triplet forces of every triplet-grid cell, then (remaining workgroups)
// the pair list of every pair-grid cell.
hipError_t launch_triplet_and_list(hipStream_t st, const TripletArgs &a, const ListBuildArgs &b,
                                   bool fp32);
size_t triplet_lds_bytes(int stage_cap, int list_cap, bool fp32);
// Triplet workgroups that fit on one CU (registers, and lds bytes of dynamic LDS each out
// of lds_per_cu); -1: unknown.
int triplet_blocks_per_cu(bool fp32, bool whole, size_t lds, size_t lds_per_cu);
hipError_t launch_triplet_gather(hipStream_t st, int64_t n, const double *pf, const int *perm,
                                 double *f, int *flags);

// Fused r-RESPA update (input particle order, FP64), in Algorithm 2's order:
//   kick2:  v <- v + dt/(2m) (F2(x^{i-1}) + F2(x^i))     (previous step's F2 kick)
//   kick3:  v <- v + dt s/(2m) F3, once or twice          (end / start of an outer cycle)
//   drift:  x <- wrap(x + dt v + dt^2/(2m) F2(x^i))
// then, when drifting, the new position is scattered to the pair list's sorted order and
// compared with the position of the last list build (skin check).
struct IntArgs {
    int64_t n;
    double *x, *v;
    const double *f2prev, *f2cur, *f3;
    double c2, c3, dt, cx;
    int kick2, kick3_end, kick3_start, drift;
    int open;               // 1: open boundaries, positions are not wrapped (DirectSum)
    const SysDesc *sd;      // any grid: only the box edges are used
    const int *sys_of;
    const int *inv_perm;    // input -> sorted index of the pair grid, or null
    Pos4 *xs;               // sorted positions of the pair grid, or null
    const double *x_ref;    // positions at the last list build (pair grid order), or null
    double half_skin2;      // (skin / 2)^2
    int *flags;
};
hipError_t launch_int(hipStream_t st, const IntArgs &a);

// Energy reductions: one workgroup per system, fixed summation order.
struct ReduceArgs {
    int nsys;
    const SysDesc *sd;
    const double *v;        // [n][3] or null (K = 0)
    double half_mass;
    const double *pe;       // per-particle pair energies [n][2] or null
    const double *ce;       // per-cell triplet energies [ncell][2] or null
    const long long *cc;    // per-cell triplet counts or null
    double *out;            // [nsys][stride]
    int stride;             // 5: {K,U2,U3,W2,W3}; 2: {U,W} from whichever source is non-null
    long long *count_out;   // [nsys] triplet counts or null
    int *flags;
    int *row;               // optional device row counter: row[0] is the row to write
                            // (out += row * nsys * stride) and is advanced by one
    double *part;           // scratch [nsys][chunks][6]
    int *done;              // [nsys + 1] completion counters, zero between launches
    int chunks;             // workgroups per system in the grid, >= red_chunks(n) of each
};
// Chunks of one system's reduction: 64 per 256 Ki particles, from 64 up to 256 (each
// chunk's last block to finish takes a device atomic on one counter, so more chunks cost
// more than their shorter loops save), and a function of the system's own particle count,
// so that a system sums in the same order alone and in a batch.
constexpr int kRedChunks = 64;
constexpr int kRedChunksMax = 4 * kRedChunks;
__host__ __device__ inline int red_chunks(int64_t n) {
    const int64_t m = (n + 262143) >> 18;
    return (int)(m < 1 ? 1 : (m > 4 ? 4 : m)) * kRedChunks;
}

// ---- DirectSum (no cutoff, open boundaries)
constexpr int kDirBlock = 64;  // particles per block of the all-triplets kernel

// One workgroup of the all-triplets kernel: block triple (I <= J <= K) of system sys.
struct DirectTask {
    int sys, I, J, K;
    int j0, j1;              // the task's range of j slots in block J (a split triple)
};
// A system's block triples are split along j into this many tasks when it has too few
// triples to fill the chip (about 2,048 tasks); the split depends on the system alone, so
// batched and single handles sum the same partial slots.
constexpr int kDirTaskTarget = 2048;
constexpr int kDirMaxSplit = 8;
struct DirectArgs {
    int ntask;
    const DirectTask *task;  // [ntask], systems in order
    const SysDesc *sd;       // p0, n of each system
    const double *x;         // [N][3] positions, input order, no wrapping
    double nu;
    double *pI, *pJ, *pK;    // [ntask][3][kDirBlock] partial forces of blocks I, J and K
    double *ce;              // [ntask][2] ATM energy and virial, or null
    int nblk;                // 64-particle blocks over all systems (gather workgroups)
    const int *blk_sys;      // [nblk] system of each block
    const int *blk0;         // [nsys] first block of each system
    const int *gslot;        // per block, in summation order, the slots holding
                             // contributions to it: role (0: I, 1: J, 2: K) << 30 | task
    const int64_t *gslot0;   // [nblk + 1] offset of each block's sequence
    int *flags;
};
// All-triplets forces of every system: the triplet kernel fills the partial slots, the
// gather sums them into f ([N][3], input order).
hipError_t launch_direct_triplet(hipStream_t st, const DirectArgs &a, bool fp32, bool energy);
hipError_t launch_direct_gather(hipStream_t st, const DirectArgs &a, double *f);
struct DirectPairArgs {
    int64_t n;               // particles over all systems (one wave each)
    const int *sys_of;       // [n] system of each particle
    const SysDesc *sd;
    const double *x;
    double *f;               // [N][3]
    double *pe;              // [N][2] half of each pair's LJ energy and virial, or null
    double eps, sigma2;
    int *flags;
};
hipError_t launch_direct_pair(hipStream_t st, const DirectPairArgs &a);  // LJ in FP64
hipError_t launch_reduce(hipStream_t st, const ReduceArgs &a);
hipError_t launch_set_int(hipStream_t st, int *p, int v);  // a kernel, so it may be captured

}  // namespace mts
