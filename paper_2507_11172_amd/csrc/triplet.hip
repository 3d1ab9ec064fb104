// Axilrod-Teller-Muto triplet forces (Sec. 2.1) over every triplet whose three pairwise
// distances are all within the three-body cutoff (Sec. 4.1, Fig. 2; Sec. 4.2.2), found
// through linked cells, with Newton's third law applied across each triplet.
//
// The paper's shared-memory traversal (C01, Sec. 4.1) visits every base cell with an
// offset list of cell pairs and cannot use Newton's third law; its conclusion names
// N3-capable traversals as future work.  This kernel is such a traversal, shaped for
// CDNA wavefronts:
//
//  * Ownership.  Particles are ordered by (cell offset, lexicographic in z, y, x; then
//    slot within the cell).  A triplet belongs to its smallest member, the anchor; its
//    two partners are then "forward" of it: in the anchor cell after the anchor, or in
//    one of the 13 forward cells of the half stencil.  Every triplet is found once.
//  * One workgroup of kTripWaves wavefronts per base cell.  The base cell and its 13
//    forward cells are staged once in LDS (FP64 positions and image shifts): the
//    LDS-staged neighbour-cell tile shared by the workgroup.  Waves take anchors
//    round-robin.
//  * Per anchor (one wave):
//      A. the canonical FP64 displacement of every tile entry after the anchor and its
//         exact cutoff test, two entries per lane per round; ballot + prefix-count
//         compaction keeps the hits in tile order as the wave's list (tile index, and the
//         displacement u from the anchor with |u|^2 in FP32);
//      B. every unordered pair of list entries is tested once along the flattened
//         diagonals of the circulant (item q = (dd - 1) m + j stands for j and
//         k = (j + dd) mod m), so all lanes are busy whatever m is; the third edge j-k is
//         prefiltered in FP32 and settled, when within rounding of the cutoff, with the
//         canonical FP64 displacement; hits are compacted into a ring queue;
//      C. ATM is evaluated one queued hit per lane whenever 64 are pending, and on the
//         rest at the end of the anchor.  The FP32 form takes u from the list; the FP64
//         form recomputes it from the staged positions (the same canonical displacement,
//         so the same bits), which keeps a workgroup's LDS small enough for six per CU.
//  * Accumulation.  The partner forces of each hit go to the wave's per-list-slot FP64
//    partials by LDS atomics issued from one wave.  The order is taken to be fixed: the
//    wave's instructions reach the LDS in program order, and the lanes of one
//    instruction that hit the same address are assumed to be applied in a fixed
//    (hardware) order -- an assumption that bitwise repeat runs at 32,000 particles
//    guard.  By Newton's third law within the triplet, the anchor's force is minus the
//    sum of the partials, formed by a fixed-order wave sum.  When the anchor is done, the wave
//    merges its partials into the shared tile accumulator in anchor order, serialised by
//    a turn counter in LDS -- so the result is bitwise reproducible without float
//    atomics across waves.  At the end the tile is flushed to
//    pf[offset][component][particle]; every (offset, particle) slot has exactly one
//    writer, and the gather sums the 14 slots in fixed order.  Nothing is accumulated
//    with global float atomics.
//
// Cutoff geometry is FP64 and canonical, so the triplet set is bit-identical to the
// FP64 oracle's in both precisions; T is the precision of the ATM arithmetic.  LDS
// arrays are structure-of-arrays so that consecutive lanes touch consecutive banks.
#include <algorithm>
#include <type_traits>

#include "atm.h"
#include "common.h"
#include "list_build.h"

namespace mts {

constexpr int kTripWaves = 4;
constexpr int kTripThreads = kTripWaves * kWave;
// Hit queue: evaluated one hit per lane whenever 64 are pending; one round of tests
// (one list pair per lane: two per lane would give each lane two independent chains, but
// one keeps the registers and the queue small, which is worth more) pushes at most 64 more.
constexpr int kQueueCap = 2 * kWave;   // a ring: fewer than 64 pending + 64 pushed
constexpr int kQueueMask = kQueueCap - 1;

// Number of set bits of mask in the lanes below this one.
__device__ __forceinline__ int below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// LDS layout.  Every array has a 16-byte (or smaller) element, so that consecutive lanes
// read consecutive 16-byte words (ds_read_b128 free of bank conflicts; a 32-byte stride
// puts two of every eight lanes on the same banks): the 32-byte FP64 records are stored
// as two arrays of 16-byte halves.  Accumulators updated at scattered addresses are
// structure-of-arrays.
struct PosEnt {                // a staged particle in registers: wrapped FP64 position
    double x, y, z;            // and the image shift (0 or +-L per component) seen from
    double sx, sy, sz;         // the base cell
};

struct alignas(16) TileEnt {   // its LDS form: the stencil code of the entry's cell (a
    double x, y, z;            // 2-bit shift code per component, the cell in bits 8..)
    int code;
    int pad;
};

// Forward neighbour j of the current anchor: the canonical displacement anchor -> j and
// its square |u|^2 in the precision T of the ATM arithmetic.  The list keeps them in FP32
// (16 bytes): the j-k sweep tests in FP32, and the FP32 form evaluates from them; the
// FP64 form recomputes its FP64 entries from the tile when it evaluates a hit (32 bytes
// per entry and wave would cost the fourth workgroup per CU, which is worth more than
// the recomputation).
template <typename T>
struct alignas(16) ListEnt {
    T ux, uy, uz, a;
};

static_assert(sizeof(TileEnt) == 32 && sizeof(ListEnt<float>) == 16, "LDS entry sizes");

// A whole-system tile carries no image shifts: the shift of entry e as seen from the
// anchor is that of the minimum image, S = -L rint((x_e - x_a) / L), so that
// disp1(x_a, x_e, S) = fl(fl(x_e - x_a) + S) is the canonical displacement.
__device__ __forceinline__ void mic_from(PosEnt &e, const PosEnt &an, const SysDesc &d) {
    e.sx = -d.L[0] * rint((e.x - an.x) * d.iL[0]);
    e.sy = -d.L[1] * rint((e.y - an.y) * d.iL[1]);
    e.sz = -d.L[2] * rint((e.z - an.z) * d.iL[2]);
}

struct Tile {                  // staged neighbour cells, CAP entries
    double2 *exy;              // TileEnt halves: (x, y) and (z, shift code)
    double2 *ezc;
    double *fx, *fy, *fz;      // force accumulators
};

__device__ __forceinline__ TileEnt tile_get(const Tile &tl, int t) {
    const double2 a = tl.exy[t], b = tl.ezc[t];
    TileEnt e;
    e.x = a.x;
    e.y = a.y;
    e.z = b.x;
    e.code = (int)__double_as_longlong(b.y);
    e.pad = 0;
    return e;
}

__device__ __forceinline__ void tile_set(const Tile &tl, int t, const TileEnt &e) {
    tl.exy[t] = make_double2(e.x, e.y);
    tl.ezc[t] = make_double2(e.z, __longlong_as_double((long long)e.code));
}

struct List {                  // one wave's forward-neighbour list, LC entries
    ListEnt<float> *f;         // displacement from the anchor and its square, FP32
    double *px, *py, *pz;      // partner force partials of the current anchor
    int *t;                    // tile index
    unsigned short *q;         // hit queue, kQueueCap entries: j | k << 8 (lists <= 256)
};

// The same layout in both precisions (the argument is kept for the callers).
size_t triplet_lds_bytes(int cap, int lcap, bool /*fp32*/) {
    return (size_t)cap * (sizeof(TileEnt) + 3 * sizeof(double)) +
           (size_t)kTripWaves * lcap * (sizeof(ListEnt<float>) + 3 * sizeof(double) + sizeof(int)) +
           (size_t)kTripWaves * kQueueCap * sizeof(unsigned short);
}

// Carves the dynamic LDS block (cap is a multiple of 32 and lc of 16, so every array
// starts 16-byte aligned): 16-byte entries, then doubles, ints and the queue.
__device__ __forceinline__ void carve(unsigned char *raw, int cap, int lc, int wave, Tile &tl,
                                      List &L) {
    tl.exy = (double2 *)raw;
    tl.ezc = tl.exy + cap;
    ListEnt<float> *lf = (ListEnt<float> *)(tl.ezc + cap);
    L.f = lf + (size_t)wave * lc;
    lf += (size_t)kTripWaves * lc;
    double *dp = (double *)lf;
    tl.fx = dp; tl.fy = dp + cap; tl.fz = dp + 2 * cap;
    double *pw = dp + 3 * (size_t)cap + (size_t)wave * 3 * lc;
    L.px = pw; L.py = pw + lc; L.pz = pw + 2 * lc;
    int *ip = (int *)(dp + 3 * (size_t)cap + (size_t)kTripWaves * 3 * lc);
    L.t = ip + (size_t)wave * lc;
    L.q = (unsigned short *)(ip + (size_t)kTripWaves * lc) + (size_t)wave * kQueueCap;
}

// FP32 prefilter of the j-k cutoff test, on v = w - u from the FP32 list entries.  The
// displacements (|u| <= rc) carry FP32 errors below 1e-6 relative to rc^2 in a squared
// distance, so a relative band of 1e-5 around rc^2 separates certain hits (below),
// certain misses (above) and the rare ambiguous cases, which are settled by the canonical
// FP64 test: the triplet set is exactly the FP64 one.
constexpr float kPrefilterBand = 1e-5f;

// One queued triplet (anchor, j, k): the forces on the partners j and k (the anchor's is
// minus their sum), energy and virial.
template <typename T>
struct AtmOut {
    T fjx, fjy, fjz, fkx, fky, fkz, phi, vir;
};

template <typename T>
__device__ __forceinline__ AtmOut<T> atm_triplet(const ListEnt<T> &lj, const ListEnt<T> &lk, T nu) {
    // third edge for the force arithmetic: v = w - u (the cutoff test used the canonical
    // displacement; the two differ by rounding only)
    const T ux = lj.ux, uy = lj.uy, uz = lj.uz;
    const T wx = lk.ux, wy = lk.uy, wz = lk.uz;
    const T vx = wx - ux, vy = wy - uy, vz = wz - uz;
    const T cc = fma(vz, vz, fma(vy, vy, vx * vx));
    const T aa = lj.a, bb = lk.a;
    T phi, ga, gb, gc;
    atm_terms<T>(aa, bb, cc, nu, phi, ga, gb, gc);
    AtmOut<T> o;
    o.fjx = fma(gc, vx, -ga * ux);
    o.fjy = fma(gc, vy, -ga * uy);
    o.fjz = fma(gc, vz, -ga * uz);
    o.fkx = fma(-gb, wx, -(gc * vx));  // -(gb w + gc v), rounded once as before
    o.fky = fma(-gb, wy, -(gc * vy));
    o.fkz = fma(-gb, wz, -(gc * vz));
    o.phi = phi;
    o.vir = -fma(aa, ga, fma(bb, gb, cc * gc));
    return o;
}

// Wave-wide sum landing in lane 63, by DPP: quad swaps, half-row and row mirrors, then
// row broadcasts 15 and 31 (fixed order, so bitwise reproducible).  Returned to every
// lane through a read of lane 63.  Called with every lane active.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The same move for a permutation within each row: every lane is written from a lane of
// its own row, so the destination's previous content is not needed (no zero fill).
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum of each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_row<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_row<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_row<0x141>(v);  // row_half_mirror
    v += dpp_row<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum(v);
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return lane_value(v, 63);
}

// wave_sum when lanes 32..63 hold +0.0: lane 31 holds rows 0 and 1 summed in the same
// order, and adding the zero rows 2 and 3 would not change a bit.
__device__ __forceinline__ double wave_sum_lo(double v) {
    v = row_sum(v);
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    return lane_value(v, 31);
}

// Sorted particle index of tile entry t (debug listing only).
__device__ __forceinline__ int tile_slot(const StencilTable<kNumHalf> &tab, int t) {
    const int o = stencil_cell_of<kNumHalf>(tab, t);
    return tab.begin[o] + (t - tab.off[o]);
}

// Forward-list entries keep their tile index in the low bits of L.t; the weighted pass
// of a nested full step marks entries within the class split of the anchor with this bit.
constexpr int kInnerBit = 1 << 30;
constexpr int kTileMask = kInnerBit - 1;

// The triplet work of one base cell (one workgroup of kTripThreads threads).  A system with
// fewer than 14 cells (SysDesc.whole) is staged whole instead, with minimum-image
// displacements; its cell c then stands for the c-th of ncell chunks of anchors, each
// chunk writing partial slot c of every particle of the system.  WEIGHT: the
// full-step pass of nested r-RESPA -- each triplet's forces are scaled by 1 if its longest
// edge is within the split (a.ra2: all three squared edges <= ra2, decided exactly as the
// cutoff is) and by a.w_out otherwise, so that the slots sum to F_in + w_out F_out;
// energies and virials stay unscaled.
template <typename T, bool LIST, bool ENERGY, bool WEIGHT, bool WHOLE>
__device__ __forceinline__ void triplet_block(const TripletArgs &a, int base,
                                              unsigned char *smem_raw) {
    __shared__ int s_turn;
    __shared__ double s_anc[kTripWaves][3];  // each wave's current anchor force
    __shared__ double s_red[kTripWaves][2];
    __shared__ int s_cnt[kTripWaves];
    __shared__ StencilTable<kNumHalf> tab;
    __shared__ double2 s_sxy[kNumHalf];  // image shift of each stencil cell
    __shared__ double s_sz[kNumHalf];
    const int CAP = a.stage_cap, LC = a.list_cap;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t n = a.n;
    const int sysq = a.sys_of_cell[base];
    const SysDesc &d = a.sd[sysq];
    constexpr bool whole = WHOLE;  // d.whole != 0: the caller dispatches on it
    const int loc = base - d.cell0;
    const int cx = loc % d.nc[0], cy = (loc / d.nc[0]) % d.nc[1], cz = loc / (d.nc[0] * d.nc[1]);
    const double L0 = d.L[0], L1 = d.L[1], L2 = d.L[2];
    Tile tile;
    List L;
    carve(smem_raw, CAP, LC, wave, tile, L);

    // ---- stage the base cell and its 13 forward cells (shared by the workgroup), or the
    // whole system; anchors are the tile entries [a_lo, a_hi)
    int nst, a_lo, a_hi, p0s = 0;
    if (whole) {
        p0s = a.start[d.cell0];
        nst = a.start[d.cell0 + d.ncell] - p0s;
        a_lo = (int)((int64_t)loc * nst / d.ncell);
        a_hi = (int)((int64_t)(loc + 1) * nst / d.ncell);
    } else {
        nst = stencil_table<kNumHalf, true>(tab, d, cx, cy, cz, a.start);
        a_lo = 0;
        a_hi = tab.off[1];
    }
    if (a.stats && tid == 0) atomicMax(&a.stats[0], nst);
    if ((a.stats || nst > CAP) && tid == 0) atomicMax(&a.tile_obs[sysq], nst);
    if (nst > CAP) {
        if (tid == 0) atomicOr(a.flags, kFlagStageOverflow);
        nst = CAP;
    }
    a_hi = min(a_hi, nst);
    // workgroup-uniform: the loops over tile entries and anchors stay scalar
    nst = __builtin_amdgcn_readfirstlane(nst);
    a_lo = __builtin_amdgcn_readfirstlane(a_lo);
    a_hi = __builtin_amdgcn_readfirstlane(a_hi);
    for (int t = tid; t < nst; t += kTripThreads) {
        int src, code;
        if (whole) {
            src = p0s + t;
            code = 0x15;  // zero shift code: images follow the anchor (mic_from)
        } else {
            const int o = stencil_cell_of<kNumHalf>(tab, t);
            src = tab.begin[o] + (t - tab.off[o]);
            code = tab.code[o];
        }
        const Pos4 ps = a.xs[src];
        TileEnt te;
        te.x = ps.x;
        te.y = ps.y;
        te.z = ps.z;
        te.code = code;
        te.pad = 0;
        tile_set(tile, t, te);
        tile.fx[t] = 0.0;
        tile.fy[t] = 0.0;
        tile.fz[t] = 0.0;
    }
    // image shift (c - 1) L of each stencil cell from its 2-bit codes c (c L - L is exact
    // for c in {0, 1, 2}); a tile entry carries its cell in code >> 8.  Whole-system
    // tiles: no shift (the minimum image is taken per pair)
    if (tid < kNumHalf) {
        const int c = whole ? 0x15 : tab.code[tid];
        s_sxy[tid] = make_double2(fma((double)(unsigned)(c & 3), L0, -L0),
                                  fma((double)(unsigned)((c >> 2) & 3), L1, -L1));
        s_sz[tid] = fma((double)(unsigned)((c >> 4) & 3), L2, -L2);
    }
    if (tid == 0) s_turn = a_lo;
    __syncthreads();
    auto unpack_s = [&](const TileEnt &t) {
        PosEnt e;
        e.x = t.x;
        e.y = t.y;
        e.z = t.z;
        const int o = t.code >> 8;
        const double2 sxy = s_sxy[o];
        e.sx = sxy.x;
        e.sy = sxy.y;
        e.sz = s_sz[o];
        return e;
    };

    const T nu = (T)a.nu;
    const double rc2 = a.rc2;
    const float jk_lo = (float)rc2 * (1.0f - kPrefilterBand);
    const float jk_hi = (float)rc2 * (1.0f + kPrefilterBand);
    unsigned short *Q = L.q;
    double U = 0.0, W = 0.0;
    int ntrip = 0;  // wave-uniform
    auto tix = [](int v) {
        if constexpr (WEIGHT) return v & kTileMask;
        else return v;
    };
    const double ra2 = a.ra2;

    // sorted particle index of tile entry t (debug listing only)
    auto slot_of = [&](int t) { return whole ? p0s + t : tile_slot(tab, t); };
    for (int ia = a_lo + wave; ia < a_hi; ia += kTripWaves) {
        const PosEnt an = unpack_s(tile_get(tile, ia));  // anchor: base cell, zero shift
        auto entry = [&](int t) {  // tile entry t with its image shift seen from the anchor
            PosEnt e = unpack_s(tile_get(tile, t));
            if (whole) mic_from(e, an, d);
            return e;
        };
        // list entry j in the precision of the ATM arithmetic: FP32 from the list, FP64
        // recomputed from the tile (the canonical displacement of step A, bit for bit)
        auto list_entry = [&](int j) {
            if constexpr (sizeof(T) == sizeof(float)) {
                return L.f[j];
            } else {
                const PosEnt e = entry(tix(L.t[j]));
                const double dx = disp1(an.x, e.x, e.sx), dy = disp1(an.y, e.y, e.sy),
                             dz = disp1(an.z, e.z, e.sz);
                return ListEnt<T>{dx, dy, dz, norm2(dx, dy, dz)};
            }
        };
        // ---- A: canonical FP64 displacement and exact test of the tile entries after the
        // anchor, two per lane per round; ballot + prefix-count compaction keeps tile order
        int m = 0;
        {
            for (int t0 = ia + 1; t0 < nst; t0 += 2 * kWave) {
                const int t1 = t0 + lane, t2 = t0 + kWave + lane;
                const PosEnt e1 = entry(t1 < nst ? t1 : ia);
                const PosEnt e2 = entry(t2 < nst ? t2 : ia);
                const double x1 = disp1(an.x, e1.x, e1.sx), y1 = disp1(an.y, e1.y, e1.sy),
                             z1 = disp1(an.z, e1.z, e1.sz);
                const double x2 = disp1(an.x, e2.x, e2.sx), y2 = disp1(an.y, e2.y, e2.sy),
                             z2 = disp1(an.z, e2.z, e2.sz);
                const double q1 = norm2(x1, y1, z1), q2 = norm2(x2, y2, z2);
                const bool in1 = t1 < nst && q1 <= rc2;
                const bool in2 = t2 < nst && q2 <= rc2;
                // the masks from the compares themselves (a ballot of their conjunction
                // would first be materialised in a vector register)
                const uint64_t m1 = ballot(t1 < nst) & ballot(q1 <= rc2);
                const uint64_t m2 = ballot(t2 < nst) & ballot(q2 <= rc2);
                const int n1 = __popcll(m1);
                const int p1 = m + below(m1), p2 = m + n1 + below(m2);
                if (in1 && p1 < LC) {
                    L.f[p1] = ListEnt<float>{(float)x1, (float)y1, (float)z1, (float)q1};
                    L.t[p1] = WEIGHT && q1 <= ra2 ? (t1 | kInnerBit) : t1;
                    L.px[p1] = 0.0;
                    L.py[p1] = 0.0;
                    L.pz[p1] = 0.0;
                }
                if (in2 && p2 < LC) {
                    L.f[p2] = ListEnt<float>{(float)x2, (float)y2, (float)z2, (float)q2};
                    L.t[p2] = WEIGHT && q2 <= ra2 ? (t2 | kInnerBit) : t2;
                    L.px[p2] = 0.0;
                    L.py[p2] = 0.0;
                    L.pz[p2] = 0.0;
                }
                m += n1 + __popcll(m2);
            }
            if (a.stats && lane == 0) atomicMax(&a.stats[1], m);
            if (m > LC) {
                if (lane == 0) atomicOr(a.flags, kFlagListOverflow);
                m = LC;
            }
        }
        __builtin_amdgcn_wave_barrier();

        // ---- B + C: j-k tests, queued hits evaluated two per lane
        int qh = 0, qt = 0;  // ring queue head and tail (wave-uniform)
        auto scatter = [&](const AtmOut<T> &o, int j, int k) {
            atomicAdd(&L.px[j], (double)o.fjx);
            atomicAdd(&L.py[j], (double)o.fjy);
            atomicAdd(&L.pz[j], (double)o.fjz);
            atomicAdd(&L.px[k], (double)o.fkx);
            atomicAdd(&L.py[k], (double)o.fky);
            atomicAdd(&L.pz[k], (double)o.fkz);
            if (LIST) {
                const long long sidx = (long long)atomicAdd(a.list_n, 1ull);
                if (sidx < a.list_rows) {
                    const int p0 = a.perm[slot_of(ia)];
                    const int p1 = a.perm[slot_of(tix(L.t[j]))];
                    const int p2 = a.perm[slot_of(tix(L.t[k]))];
                    const int lo = min(p0, min(p1, p2)), hi = max(p0, max(p1, p2));
                    a.list_ijk[3 * sidx] = lo;
                    a.list_ijk[3 * sidx + 1] = p0 + p1 + p2 - lo - hi;
                    a.list_ijk[3 * sidx + 2] = hi;
                }
            }
        };
        // Class of a hit (WEIGHT): inner iff both anchor edges were within the split at the
        // list build (exact FP64 test, kInnerBit) and so is the j-k edge: from the list
        // displacements, settled by the canonical FP64 displacement within a band around
        // the split that covers their rounding (rare).
        const T nu_out = (T)(a.nu * a.w_out);
        const double inv_w = 1.0 / a.w_out;
        const double band = (sizeof(T) == sizeof(float) ? 1e-5 : 1e-12) * rc2;
        auto inner_class = [&](int j, int k, const ListEnt<T> &uj, const ListEnt<T> &uk) {
            const int tj = L.t[j], tk = L.t[k];
            bool in = (tj & tk & kInnerBit) != 0;
            const T vx = uk.ux - uj.ux, vy = uk.uy - uj.uy, vz = uk.uz - uj.uz;
            const double c = (double)((vx * vx + vy * vy) + vz * vz);
            const bool amb = in && c > ra2 - band && c <= ra2 + band;
            in = in && c <= ra2 - band;
            if (ballot(amb)) {
                if (amb) {
                    const PosEnt ej = entry(tj & kTileMask);
                    const PosEnt ek = entry(tk & kTileMask);
                    const double wx = disp1(ej.x, ek.x, ek.sx - ej.sx);
                    const double wy = disp1(ej.y, ek.y, ek.sy - ej.sy);
                    const double wz = disp1(ej.z, ek.z, ek.sz - ej.sz);
                    in = norm2(wx, wy, wz) <= ra2;
                }
            }
            return in;
        };
        // One queued hit per lane (lanes without one compute on the first pending entry and
        // are masked): the forces on j and k go to the list partials; the anchor's force is
        // not formed here -- by Newton's third law within the triplet it is minus the sum
        // of the partner forces, and the merge takes it from the partials.
        auto evaluate = [&](int cnt) {
            const bool v1 = lane < cnt;
            const int e1 = Q[(qh + (v1 ? lane : 0)) & kQueueMask];
            qh += cnt;
            const int j1 = e1 & 0xff, k1 = e1 >> 8;
            const ListEnt<T> uj1 = list_entry(j1), uk1 = list_entry(k1);
            T nu1 = nu;
            double iw1 = 1.0;  // unscales the energy terms of weighted triplets
            if constexpr (WEIGHT) {
                const bool in1 = inner_class(j1, k1, uj1, uk1);
                nu1 = in1 ? nu : nu_out;
                iw1 = in1 ? 1.0 : inv_w;
            }
            const AtmOut<T> o1 = atm_triplet<T>(uj1, uk1, nu1);
            if (ENERGY) {
                U += v1 ? (double)o1.phi * iw1 : 0.0;
                W += v1 ? (double)o1.vir * iw1 : 0.0;
            }
            if (v1) scatter(o1, j1, k1);
            __builtin_amdgcn_wave_barrier();
        };

        // ---- B: the j-k test of every unordered list pair, one per lane and round.
        // Pair item q = (dd - 1) m + j stands for (j, k = (j + dd) mod m): diagonals
        // dd = 1, 2, ... of the circulant, each a permutation of the list; for even m the
        // last diagonal dd = m/2 pairs each entry with its opposite, and its first half
        // (j < m/2) covers those pairs once, so q < m(m - 1)/2 visits every pair exactly
        // once with all lanes busy.  Lane l takes q = l and advances by 64.
        m = __builtin_amdgcn_readfirstlane(m);  // wave-uniform: keeps m and what follows scalar
        const int npair = m * (m - 1) / 2;
        if (npair > 0) {
            // 64 = adv_d m + adv_j, and item q = (dd - 1) m + j: quotients from the
            // hardware reciprocal of m, corrected by one step where it rounded across.
            // An advance by 64 items moves j by adv_j mod m, and dd by adv_d plus the carry
            // of j's wrap, so k = (j + dd) mod m moves by (adv_j + adv_d) mod m plus that
            // carry; with more than one round m >= 12 and adv_d <= 5 < m, so each sum is
            // below 2m and one conditional subtraction reduces it: (j + a) mod m for
            // j + a < 2m is min(j + a, j + a - m) in unsigned arithmetic (the second
            // wraps when j + a < m).
            const float rm = __builtin_amdgcn_rcpf((float)m);
            int adv_d = (int)((float)kWave * rm), adv_j = kWave - adv_d * m;
            if (adv_j >= m) { adv_j -= m; ++adv_d; }
            if (adv_j < 0) { adv_j += m; --adv_d; }
            int adv_k = adv_j + adv_d;
            if (adv_k >= m) adv_k -= m;
            const unsigned aj = (unsigned)__builtin_amdgcn_readfirstlane(adv_j);
            const unsigned ak = (unsigned)__builtin_amdgcn_readfirstlane(adv_k);
            const unsigned um = (unsigned)m;
            unsigned jj, kk;
            {  // (j, k) of item lane
                int d0 = (int)(((float)lane + 0.5f) * rm);
                int j0 = lane - d0 * m;
                if (j0 >= m) { j0 -= m; ++d0; }
                if (j0 < 0) { j0 += m; --d0; }
                int k0 = j0 + d0 + 1;   // dd <= m/2 for a valid item: one step
                k0 -= k0 >= m ? m : 0;
                jj = (unsigned)j0;
                kk = (unsigned)k0;
            }
            // the canonical FP64 test of a j-k edge within rounding of the cutoff (rare)
            auto settle = [&](int j, int k) {
                const PosEnt ej = entry(tix(L.t[j]));
                const PosEnt ek = entry(tix(L.t[k]));
                const double wx = disp1(ej.x, ek.x, ek.sx - ej.sx);
                const double wy = disp1(ej.y, ek.y, ek.sy - ej.sy);
                const double wz = disp1(ej.z, ek.z, ek.sz - ej.sz);
                return norm2(wx, wy, wz) <= rc2;
            };
            for (int q0 = 0; q0 < npair; q0 += kWave) {
                // FP32 |u_k - u_j|^2 of this lane's item; the round that runs past the
                // last item (CHECK) gives its idle lanes +inf and reads entry 0 for them
                auto jk2 = [&](auto check) {
                    constexpr bool CHECK = decltype(check)::value;
                    const bool ok = !CHECK || q0 + lane < npair;
                    const ListEnt<float> fj = L.f[CHECK && !ok ? 0u : jj];
                    const ListEnt<float> fk = L.f[CHECK && !ok ? 0u : kk];
                    const float x = fk.ux - fj.ux, y = fk.uy - fj.uy, z = fk.uz - fj.uz;
                    const float c = fmaf(z, z, fmaf(y, y, x * x));
                    return CHECK && !ok ? __builtin_inff() : c;
                };
                float c;
                if (q0 + kWave <= npair) c = jk2(std::false_type{});
                else c = jk2(std::true_type{});
                bool hit = c <= jk_lo;
                uint64_t mh = ballot(hit);
                if (ballot(c <= jk_hi) & ~mh) {  // rare: settle with the canonical FP64 test
                    bool s = false;
                    if (c > jk_lo && c <= jk_hi) s = settle((int)jj, (int)kk);
                    hit = hit || s;
                    mh |= ballot(s);
                }
                // append the hits to the ring queue in lane order
                if (hit) Q[(qt + below(mh)) & kQueueMask] = (unsigned short)(jj | (kk << 8));
                qt += __popcll(mh);
                __builtin_amdgcn_wave_barrier();
                while (qt - qh >= kWave) {
                    evaluate(kWave);
                    ntrip += kWave;
                }
                const unsigned j1 = jj + aj, k1 = kk + ak + (j1 >= um ? 1u : 0u);
                jj = min(j1, j1 - um);
                kk = min(k1, k1 - um);
            }
            if (qt > qh) {
                ntrip += qt - qh;
                evaluate(qt - qh);
            }
        }

        // ---- the anchor's force: minus the sum of its partners' partials (a fixed-order
        // wave sum)
        double *anc = s_anc[wave];
        {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int t = lane; t < m; t += kWave) {
                sx -= L.px[t];
                sy -= L.py[t];
                sz -= L.pz[t];
            }
            if (m <= 32) {  // lanes from m on hold +0.0 and none holds -0.0: rows 2, 3 add nothing
                sx = wave_sum_lo(sx);
                sy = wave_sum_lo(sy);
                sz = wave_sum_lo(sz);
            } else {
                sx = wave_sum(sx);
                sy = wave_sum(sy);
                sz = wave_sum(sz);
            }
            if (lane == 0) {
                anc[0] = sx;
                anc[1] = sy;
                anc[2] = sz;
            }
        }
        // ---- merge this anchor's forces into the tile, in anchor order
        if (lane == 0) {
            while (__hip_atomic_load(&s_turn, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != ia)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int t = lane; t < m; t += kWave) {
            const int te = tix(L.t[t]);
            tile.fx[te] += L.px[t];
            tile.fy[te] += L.py[t];
            tile.fz[te] += L.pz[t];
        }
        if (lane < 3) {
            double *f = lane == 0 ? tile.fx : (lane == 1 ? tile.fy : tile.fz);
            f[ia] += anc[lane];
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) __hip_atomic_store(&s_turn, ia + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (ENERGY) {
        U = wave_sum(U);
        W = wave_sum(W);
    }
    if (lane == 0) {
        s_red[wave][0] = U;
        s_red[wave][1] = W;
        s_cnt[wave] = ntrip;
    }
    __syncthreads();

    // ---- flush the tile's forces: slot (offset, particle) has exactly one writer; a
    // whole-system chunk c writes slot c of every particle of the system, chunk 0 also
    // clears the slots no chunk uses
    if (whole) {
        for (int t = tid; t < nst; t += kTripThreads) {
            const int64_t p = p0s + t;
            a.pf[(3 * loc) * n + p] = tile.fx[t];
            a.pf[(3 * loc + 1) * n + p] = tile.fy[t];
            a.pf[(3 * loc + 2) * n + p] = tile.fz[t];
        }
        if (loc == 0)
            for (int o = d.ncell; o < kNumHalf; ++o)
                for (int t = tid; t < nst; t += kTripThreads)
                    for (int k = 0; k < 3; ++k) a.pf[(3 * o + k) * n + p0s + t] = 0.0;
    } else {
        for (int t = tid; t < nst; t += kTripThreads) {
            const int o = stencil_cell_of<kNumHalf>(tab, t);
            const int64_t p = tab.begin[o] + (t - tab.off[o]);
            a.pf[(3 * o) * n + p] = tile.fx[t];
            a.pf[(3 * o + 1) * n + p] = tile.fy[t];
            a.pf[(3 * o + 2) * n + p] = tile.fz[t];
        }
    }
    if (tid == 0) {
        long long c = 0;
        for (int q = 0; q < kTripWaves; ++q) c += s_cnt[q];
        if (a.cc) a.cc[base] = c;
        if (ENERGY) {
            double u = 0.0, w = 0.0;
            for (int q = 0; q < kTripWaves; ++q) {
                u += s_red[q][0];
                w += s_red[q][1];
            }
            a.ce[2 * base] = u;
            a.ce[2 * base + 1] = w;
        }
    }
}

// Sum of the 14 partial slots of every particle, written in input order.
__global__ void __launch_bounds__(256) k_triplet_gather(int64_t n, const double *__restrict__ pf,
                                                        const int *__restrict__ perm,
                                                        double *__restrict__ f, int *flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < kNumHalf; ++o) {
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] += pf[(3 * o + k) * n + p];
    }
    const int64_t i = perm[p];
    f[3 * i] = s[0];
    f[3 * i + 1] = s[1];
    f[3 * i + 2] = s[2];
    if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2])) atomicOr(flags, kFlagNonFinite);
}

// One launch per force evaluation over the items of every system: workgroup b takes the
// triplet base cell a.cell_map[b] (the host orders the cells by decreasing estimated
// work, so the dispatcher starts the costly ones first), and the workgroups past the
// a.ncell triplet items build the pair list of one pair-grid cell each, filling the
// compute units that the triplet items leave idle as they drain.  (A persistent form
// that pops items from a device counter was measured 20-25 % slower: the dispatcher
// overlaps the start of one workgroup with the tail of another on a compute unit.)
//   LB: the launch also builds the pair list; WH: some system is staged whole (the whole-
//   system code path costs registers, so launches without such systems leave it out).
// OCC: waves per SIMD the registers are held to.  Five (96 VGPRs) let five workgroups
// share a CU when tiles and lists fit 32 KB of LDS (1M particles, FP64: 3.0 -> 2.7 ms;
// the whole-system weighted variant spills a few registers for it); six (80 VGPRs; the
// variants with whole-system tiles spill a few) pay only when the LDS also admits six
// workgroups, so the launcher takes them exactly then (TripletArgs.occ6).
template <typename T, bool LIST, bool ENERGY, bool WEIGHT, bool LB, bool WH, int OCC>
__global__ void __launch_bounds__(kTripThreads) __attribute__((amdgpu_waves_per_eu(OCC)))
k_triplet_items(TripletArgs a, ListBuildArgs b) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int it = (int)blockIdx.x;
    if (it < a.ncell) {
        const int base = a.cell_map ? a.cell_map[it] : it;
        if (WH && a.sd[a.sys_of_cell[base]].whole)
            triplet_block<T, LIST, ENERGY, WEIGHT, WH>(a, base, smem_raw);
        else
            triplet_block<T, LIST, ENERGY, WEIGHT, false>(a, base, smem_raw);
    } else if constexpr (LB) {
        list_build_block(b, it - a.ncell, smem_raw);
    }
}

template <typename T, bool LIST, bool ENERGY, bool WEIGHT, int OCC>
static void launch_items_o(hipStream_t st, const TripletArgs &a, const ListBuildArgs &b,
                           size_t lds, int grid) {
    if (b.ncell > 0) {
        if constexpr (!LIST) {
            if (a.any_whole) k_triplet_items<T, LIST, ENERGY, WEIGHT, true, true, OCC><<<grid, kTripThreads, lds, st>>>(a, b);
            else k_triplet_items<T, LIST, ENERGY, WEIGHT, true, false, OCC><<<grid, kTripThreads, lds, st>>>(a, b);
        }
    } else {
        if (a.any_whole) k_triplet_items<T, LIST, ENERGY, WEIGHT, false, true, OCC><<<grid, kTripThreads, lds, st>>>(a, b);
        else k_triplet_items<T, LIST, ENERGY, WEIGHT, false, false, OCC><<<grid, kTripThreads, lds, st>>>(a, b);
    }
}

template <typename T, bool LIST, bool ENERGY, bool WEIGHT>
static hipError_t launch_items_t(hipStream_t st, const TripletArgs &a, const ListBuildArgs &b) {
    size_t lds = a.ncell > 0 ? triplet_lds_bytes(a.stage_cap, a.list_cap, sizeof(T) == 4) : 0;
    if (b.ncell > 0) lds = std::max(lds, list_build_bytes(b.stage_cap));
    const int grid = a.ncell + b.ncell;
    if constexpr (!LIST && !WEIGHT) {  // the plain passes come in both register budgets
        if (a.occ6) {
            launch_items_o<T, LIST, ENERGY, WEIGHT, 6>(st, a, b, lds, grid);
            return hipGetLastError();
        }
    }
    launch_items_o<T, LIST, ENERGY, WEIGHT, 5>(st, a, b, lds, grid);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_items_p(hipStream_t st, const TripletArgs &a, const ListBuildArgs &b,
                                 bool listing) {
    if (listing) return launch_items_t<T, true, false, false>(st, a, b);
    if (a.w_out > 1.0)
        return a.ce ? launch_items_t<T, false, true, true>(st, a, b)
                    : launch_items_t<T, false, false, true>(st, a, b);
    return a.ce ? launch_items_t<T, false, true, false>(st, a, b)
                : launch_items_t<T, false, false, false>(st, a, b);
}

hipError_t launch_triplet_and_list(hipStream_t st, const TripletArgs &a, const ListBuildArgs &b,
                                   bool fp32) {
    if (a.ncell + b.ncell <= 0) return hipSuccess;
    return fp32 ? launch_items_p<float>(st, a, b, false) : launch_items_p<double>(st, a, b, false);
}

hipError_t launch_triplet(hipStream_t st, const TripletArgs &a, bool fp32, bool listing) {
    if (a.ncell <= 0) return hipSuccess;
    const ListBuildArgs none{};
    return fp32 ? launch_items_p<float>(st, a, none, listing)
                : launch_items_p<double>(st, a, none, listing);
}

hipError_t configure_triplet_lds(size_t max_bytes) {
#define MTS_ITEMS(T, LB, WH)                                                 \
    (const void *)k_triplet_items<T, false, false, false, LB, WH, 5>,        \
        (const void *)k_triplet_items<T, false, true, false, LB, WH, 5>,     \
        (const void *)k_triplet_items<T, false, false, true, LB, WH, 5>,     \
        (const void *)k_triplet_items<T, false, true, true, LB, WH, 5>,      \
        (const void *)k_triplet_items<T, false, false, false, LB, WH, 6>,    \
        (const void *)k_triplet_items<T, false, true, false, LB, WH, 6>
    const void *fns[] = {(const void *)k_triplet_items<double, true, false, false, false, false, 5>,
                         (const void *)k_triplet_items<double, true, false, false, false, true, 5>,
                         (const void *)k_triplet_items<float, true, false, false, false, false, 5>,
                         (const void *)k_triplet_items<float, true, false, false, false, true, 5>,
                         MTS_ITEMS(double, false, false), MTS_ITEMS(double, true, false),
                         MTS_ITEMS(double, false, true), MTS_ITEMS(double, true, true),
                         MTS_ITEMS(float, false, false), MTS_ITEMS(float, true, false),
                         MTS_ITEMS(float, false, true), MTS_ITEMS(float, true, true)};
#undef MTS_ITEMS
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int triplet_blocks_per_cu(bool fp32, bool whole, size_t lds, size_t lds_per_cu) {
    auto blocks = [&](const void *f) {
        int nb = 0;
        hipFuncAttributes fa{};
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kTripThreads, 0) != hipSuccess ||
            hipFuncGetAttributes(&fa, f) != hipSuccess) {
            (void)hipGetLastError();  // leave no sticky error for the next launch check
            return -1;
        }
        // LDS goes out in granules: static + dynamic bytes rounded up to 512, plus 512 of
        // margin for a coarser granule
        const size_t per = (fa.sharedSizeBytes + lds + 511) / 512 * 512 + 512;
        return std::min(nb, (int)(lds_per_cu / per));
    };
    // the variant with the most registers of each precision and kind of launch in each
    // register budget; six per CU only where the six-wave budget reaches it
    const void *f5 =
        fp32 ? (whole ? (const void *)k_triplet_items<float, false, true, true, true, true, 5>
                      : (const void *)k_triplet_items<float, false, true, true, true, false, 5>)
             : (whole ? (const void *)k_triplet_items<double, false, true, true, true, true, 5>
                      : (const void *)k_triplet_items<double, false, true, true, true, false, 5>);
    const void *f6 =
        fp32 ? (whole ? (const void *)k_triplet_items<float, false, true, false, true, true, 6>
                      : (const void *)k_triplet_items<float, false, true, false, true, false, 6>)
             : (whole ? (const void *)k_triplet_items<double, false, true, false, true, true, 6>
                      : (const void *)k_triplet_items<double, false, true, false, true, false, 6>);
    const int n5 = blocks(f5), n6 = blocks(f6);
    if (n5 < 0) return n5;
    return n6 >= 6 ? n6 : n5;
}

hipError_t launch_triplet_gather(hipStream_t st, int64_t n, const double *pf, const int *perm,
                                 double *f, int *flags) {
    if (n > 0) k_triplet_gather<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, pf, perm, f, flags);
    return hipGetLastError();
}

}  // namespace mts
