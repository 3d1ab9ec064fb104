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
//      A. filter the tile to the anchor's forward neighbours within rc3 -- ballot +
//         prefix-count compaction into the wave's list (tile index, displacement u from
//         the anchor, |u|^2);
//      B. each lane owns one list entry j (kept in registers) and walks its partners
//         k = j + 1 .. j + m/2 around the list, so all m(m-1)/2 pairs are visited once
//         with balanced lanes; the third edge j-k is tested with the canonical FP64
//         displacement and hits are compacted into a queue;
//      C. evaluate ATM on full waves of queued hits.
//  * Accumulation.  The anchor's force stays in registers and is summed across the wave
//    with DPP row operations; partner forces go to the wave's per-list-slot FP64
//    partials (LDS atomics inside one wave: a fixed order).  When the anchor is done,
//    the wave merges its partials into the shared tile accumulator in anchor order,
//    serialised by a turn counter in LDS -- so the result is bitwise reproducible
//    without float atomics across waves.  At the end the tile is flushed to
//    pf[offset][component][particle]; every (offset, particle) slot has exactly one
//    writer, and k_triplet_gather sums the 14 slots in fixed order.  Nothing is
//    accumulated with global float atomics.
//
// Cutoff geometry is FP64 and canonical, so the triplet set is bit-identical to the
// FP64 oracle's in both precisions; T is the precision of the ATM arithmetic.  LDS
// arrays are structure-of-arrays so that consecutive lanes touch consecutive banks.
#include "common.h"

namespace mts {

constexpr int kTripWaves = 4;
constexpr int kTripThreads = kTripWaves * kWave;
constexpr int kQueueCap = 2 * kWave;

// LDS layout.  Entries read by consecutive lanes are 48-byte structures read as three
// 16-byte words: an odd multiple of 16 bytes is free of bank conflicts for
// ds_read_b128 across 16 lanes.  Accumulators updated at scattered addresses are
// structure-of-arrays.
struct alignas(16) TileEnt {   // one staged particle
    double x, y, z;            // wrapped FP64 position
    double sx, sy, sz;         // image shift (0 or +-L) seen from the base cell
};

struct alignas(16) ListEnt {   // one forward neighbour of the current anchor
    double ux, uy, uz, a;      // canonical displacement anchor -> partner, and |u|^2
    int t;                     // tile index
    int pad0;
    double pad1;
};

static_assert(sizeof(TileEnt) == 48 && sizeof(ListEnt) == 48, "48-byte LDS entries");

struct Tile {                  // staged neighbour cells, CAP entries
    TileEnt *e;
    double *fx, *fy, *fz;      // force accumulators
    int *o;                    // half-stencil offset index (selects the partial slot)
    int *slot;                 // sorted particle index
};

struct List {                  // one wave's forward-neighbour list, LC entries
    ListEnt *e;
    double *px, *py, *pz;      // partner force partials of the current anchor
    int *q;                    // hit queue, kQueueCap entries: j | k << 16
};

size_t triplet_lds_bytes(int cap, int lcap) {
    return (size_t)cap * (sizeof(TileEnt) + 3 * sizeof(double) + 2 * sizeof(int)) +
           (size_t)kTripWaves * lcap * (sizeof(ListEnt) + 3 * sizeof(double)) +
           (size_t)kTripWaves * kQueueCap * sizeof(int);
}

// Carves the dynamic LDS block (cap and lc are multiples of 32, so every array starts
// 16-byte aligned): 48-byte entries, then doubles, then ints.
__device__ __forceinline__ void carve(unsigned char *raw, int cap, int lc, int wave, Tile &T,
                                      List &L) {
    T.e = (TileEnt *)raw;
    ListEnt *le = (ListEnt *)(T.e + cap);
    L.e = le + (size_t)wave * lc;
    double *dp = (double *)(le + (size_t)kTripWaves * lc);
    T.fx = dp; T.fy = dp + cap; T.fz = dp + 2 * cap;
    double *pw = dp + 3 * (size_t)cap + (size_t)wave * 3 * lc;
    L.px = pw; L.py = pw + lc; L.pz = pw + 2 * lc;
    int *ip = (int *)(dp + 3 * (size_t)cap + (size_t)kTripWaves * 3 * lc);
    T.o = ip; T.slot = ip + cap;
    L.q = ip + 2 * cap + (size_t)wave * kQueueCap;
}

// 1/sqrt(x): hardware estimate refined by two Newton-Raphson steps y <- y (3 - x y^2)/2
// (quadratic convergence from the ~2^-22 estimate to below one FP64 ulp of error).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt_nr(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// ATM potential in squared edge lengths a = |u|^2, b = |w|^2, c = |v|^2 (u: anchor->j,
// w: anchor->k, v: j->k).  By the law of cosines the cosine product of Sec. 2.1 is
// t1 t2 t3 / (8abc), t1 = a+b-c, t2 = a-b+c, t3 = b+c-a, so
//   phi = nu [P^-3/2 + 3/8 T P^-5/2],  P = abc,  T = t1 t2 t3.
// Returns phi and g_a = 2 dphi/da, g_b, g_c; the forces are
//   F_anchor = g_a u + g_b w,  F_j = -g_a u + g_c v,  F_k = -g_b w - g_c v,
// and the triplet's virial sum_x x.F = u.F_j + w.F_k = -(a g_a + b g_b + c g_c).
template <typename T>
__device__ __forceinline__ void atm_terms(T a, T b, T c, T nu, T &phi, T &ga, T &gb, T &gc) {
    const T P = a * b * c;
    const T rs = rsqrt_t<T>(P);       // P^-1/2
    const T ip = rs * rs;             // P^-1
    const T p32 = rs * ip;            // P^-3/2
    const T p52 = p32 * ip;           // P^-5/2
    const T t1 = a + b - c, t2 = a - b + c, t3 = b + c - a;
    const T tt = t1 * t2 * t3;
    const T q = T(0.375) * p52;
    const T K = fma(T(-0.9375) * tt, p52, T(-1.5) * p32);
    const T Kp = K * ip;              // K / P;  K/a = Kp * b * c
    const T two_nu = T(2) * nu;
    ga = two_nu * fma(Kp, b * c, q * fma(T(2) * a, t3, -t1 * t2));
    gb = two_nu * fma(Kp, a * c, q * fma(T(2) * b, t2, -t1 * t3));
    gc = two_nu * fma(Kp, a * b, q * fma(T(2) * c, t1, -t2 * t3));
    phi = nu * fma(q, tt, p32);
}

// Wave-wide sum landing in lane 63, by DPP: quad swaps, half-row and row mirrors, then
// row broadcasts 15 and 31 (fixed order, so bitwise reproducible).  Returned to every
// lane through a read of lane 63.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_d<0x140, 0xf>(v);  // row_mirror
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wave_sum_int(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return __builtin_amdgcn_readlane(v, 63);
}

template <typename T, bool LIST>
__global__ void __launch_bounds__(kTripThreads) k_triplet(TripletArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ int s_turn;
    __shared__ double s_red[kTripWaves][2];
    __shared__ int s_cnt[kTripWaves];
    __shared__ StencilTable<kNumHalf> tab;
    const int CAP = a.stage_cap, LC = a.list_cap;
    const int base = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    const int64_t n = a.n;
    const SysDesc &d = a.sd[a.sys_of_cell[base]];
    const int loc = base - d.cell0;
    const int cx = loc % d.nc[0], cy = (loc / d.nc[0]) % d.nc[1], cz = loc / (d.nc[0] * d.nc[1]);
    const double L0 = d.L[0], L1 = d.L[1], L2 = d.L[2];
    Tile tile;
    List L;
    carve(smem_raw, CAP, LC, wave, tile, L);

    // ---- stage the base cell and its 13 forward cells (shared by the workgroup)
    int nst = stencil_table<kNumHalf, true>(tab, d, cx, cy, cz, a.start);
    int nself = tab.off[1];
    if (nst > CAP) {
        if (tid == 0) atomicOr(a.flags, kFlagStageOverflow);
        nst = CAP;
    }
    nself = min(nself, nst);
    for (int t = tid; t < nst; t += kTripThreads) {
        const int o = stencil_cell_of<kNumHalf>(tab, t);
        const int src = tab.begin[o] + (t - tab.off[o]);
        const int code = tab.code[o];
        const Pos4 ps = a.xs[src];
        TileEnt e;
        e.x = ps.x;
        e.y = ps.y;
        e.z = ps.z;
        e.sx = (double)((code & 3) - 1) * L0;
        e.sy = (double)(((code >> 2) & 3) - 1) * L1;
        e.sz = (double)(((code >> 4) & 3) - 1) * L2;
        tile.e[t] = e;
        tile.o[t] = code >> 8;
        tile.slot[t] = src;
        tile.fx[t] = 0.0;
        tile.fy[t] = 0.0;
        tile.fz[t] = 0.0;
    }
    if (tid == 0) s_turn = 0;
    __syncthreads();

    const T nu = (T)a.nu;
    const double rc2 = a.rc2;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    int *Q = L.q;
    double U = 0.0, W = 0.0;
    int ntrip = 0;

    for (int ia = wave; ia < nself; ia += kTripWaves) {
        const TileEnt an = tile.e[ia];  // anchor: base cell, zero shift
        // ---- A: forward neighbours of the anchor within rc3 (tile order > ia)
        int m = 0;
        for (int t0 = ia + 1; t0 < nst; t0 += kWave) {
            const int t = t0 + lane;
            bool in = false;
            double dx = 0, dy = 0, dz = 0, r2 = 0;
            if (t < nst) {
                const TileEnt e = tile.e[t];
                dx = disp1(an.x, e.x, e.sx);
                dy = disp1(an.y, e.y, e.sy);
                dz = disp1(an.z, e.z, e.sz);
                r2 = norm2(dx, dy, dz);
                in = r2 <= rc2;
            }
            const uint64_t mask = __ballot(in);
            const int pos = m + __popcll(mask & lt_mask);
            if (in && pos < LC) {
                ListEnt le;
                le.ux = dx;
                le.uy = dy;
                le.uz = dz;
                le.a = r2;
                le.t = t;
                le.pad0 = 0;
                le.pad1 = 0.0;
                L.e[pos] = le;
                L.px[pos] = 0.0;
                L.py[pos] = 0.0;
                L.pz[pos] = 0.0;
            }
            m += __popcll(mask);
        }
        if (m > LC) {
            if (lane == 0) atomicOr(a.flags, kFlagListOverflow);
            m = LC;
        }
        __builtin_amdgcn_wave_barrier();

        // ---- B + C
        double fax = 0.0, fay = 0.0, faz = 0.0;
        int qn = 0;
        auto evaluate = [&](int cnt) {
            if (lane < cnt) {
                const int e = Q[lane];
                const int j = e & 0xffff, k = e >> 16;
                const ListEnt lj = L.e[j], lk = L.e[k];
                const double uxd = lj.ux, uyd = lj.uy, uzd = lj.uz, ad = lj.a;
                const double wxd = lk.ux, wyd = lk.uy, wzd = lk.uz, bd = lk.a;
                // third edge for the force arithmetic: v = w - u (the cutoff test used the
                // canonical displacement; the two differ by rounding only)
                const T ux = (T)uxd, uy = (T)uyd, uz = (T)uzd;
                const T wx = (T)wxd, wy = (T)wyd, wz = (T)wzd;
                const T vx = wx - ux, vy = wy - uy, vz = wz - uz;
                const T cc = (vx * vx + vy * vy) + vz * vz;
                const T aa = (T)ad, bb = (T)bd;
                T phi, ga, gb, gc;
                atm_terms<T>(aa, bb, cc, nu, phi, ga, gb, gc);
                const T fix = fma(ga, ux, gb * wx), fiy = fma(ga, uy, gb * wy),
                        fiz = fma(ga, uz, gb * wz);
                const T fjx = fma(gc, vx, -ga * ux), fjy = fma(gc, vy, -ga * uy),
                        fjz = fma(gc, vz, -ga * uz);
                const T fkx = -(fix + fjx), fky = -(fiy + fjy), fkz = -(fiz + fjz);
                fax += (double)fix;
                fay += (double)fiy;
                faz += (double)fiz;
                atomicAdd(&L.px[j], (double)fjx);
                atomicAdd(&L.py[j], (double)fjy);
                atomicAdd(&L.pz[j], (double)fjz);
                atomicAdd(&L.px[k], (double)fkx);
                atomicAdd(&L.py[k], (double)fky);
                atomicAdd(&L.pz[k], (double)fkz);
                U += (double)phi;
                W -= (double)fma(aa, ga, fma(bb, gb, cc * gc));
                ++ntrip;
                if (LIST) {
                    const long long s = (long long)atomicAdd(a.list_n, 1ull);
                    if (s < a.list_rows) {
                        const int p0 = a.perm[tile.slot[ia]], p1 = a.perm[tile.slot[lj.t]],
                                  p2 = a.perm[tile.slot[lk.t]];
                        const int lo = min(p0, min(p1, p2)), hi = max(p0, max(p1, p2));
                        a.list_ijk[3 * s] = lo;
                        a.list_ijk[3 * s + 1] = p0 + p1 + p2 - lo - hi;
                        a.list_ijk[3 * s + 2] = hi;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        };
        auto push = [&](bool hit, int j, int k) {
            const uint64_t mask = __ballot(hit);
            if (hit) Q[qn + __popcll(mask & lt_mask)] = j | (k << 16);
            qn += __popcll(mask);
            __builtin_amdgcn_wave_barrier();
            if (qn >= kWave) {
                evaluate(kWave);
                qn -= kWave;
                int rest = 0;
                if (lane < qn) rest = Q[kWave + lane];
                __builtin_amdgcn_wave_barrier();
                if (lane < qn) Q[lane] = rest;
                __builtin_amdgcn_wave_barrier();
            }
        };

        if (m >= 2) {
            const int D = m >> 1;
            const bool even = (m & 1) == 0;
            // Lane -> (j, phase): with P = max(1, 64 / m) phases, lane l takes entry
            // j = jb + l % span and circular distances dd = 1 + phase, 1 + phase + P, ...
            const int P = m < kWave ? kWave / m : 1;
            const int span = m < kWave ? m : kWave;
            for (int jb = 0; jb < m; jb += span) {
                const int j = jb + lane % span;
                const int phase = lane / span;
                const bool lane_ok = phase < P && j < m;
                TileEnt ej{};
                if (lane_ok) ej = tile.e[L.e[j].t];
                for (int d0 = 1; d0 <= D; d0 += P) {
                    const int dd = d0 + phase;
                    int k = j + dd;
                    if (k >= m) k -= m;
                    bool hit = false;
                    if (lane_ok && dd <= D && !(even && dd == D && j >= D)) {
                        const TileEnt ek = tile.e[L.e[k].t];
                        const double vx = disp1(ej.x, ek.x, ek.sx - ej.sx);
                        const double vy = disp1(ej.y, ek.y, ek.sy - ej.sy);
                        const double vz = disp1(ej.z, ek.z, ek.sz - ej.sz);
                        hit = norm2(vx, vy, vz) <= rc2;
                    }
                    push(hit, j, k);
                }
            }
            if (qn > 0) evaluate(qn);
        }
        fax = wave_sum(fax);
        fay = wave_sum(fay);
        faz = wave_sum(faz);

        // ---- merge this anchor's forces into the tile, in anchor order
        if (lane == 0) {
            while (__hip_atomic_load(&s_turn, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != ia)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int t = lane; t < m; t += kWave) {
            const int te = L.e[t].t;
            tile.fx[te] += L.px[t];
            tile.fy[te] += L.py[t];
            tile.fz[te] += L.pz[t];
        }
        if (lane == 0) {
            tile.fx[ia] += fax;
            tile.fy[ia] += fay;
            tile.fz[ia] += faz;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) __hip_atomic_store(&s_turn, ia + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    U = wave_sum(U);
    W = wave_sum(W);
    ntrip = wave_sum_int(ntrip);
    if (lane == 0) {
        s_red[wave][0] = U;
        s_red[wave][1] = W;
        s_cnt[wave] = ntrip;
    }
    __syncthreads();

    // ---- flush the tile's forces: slot (offset, particle) has exactly one writer
    for (int t = tid; t < nst; t += kTripThreads) {
        const int o = tile.o[t];
        const int64_t p = tile.slot[t];
        a.pf[(3 * o) * n + p] = tile.fx[t];
        a.pf[(3 * o + 1) * n + p] = tile.fy[t];
        a.pf[(3 * o + 2) * n + p] = tile.fz[t];
    }
    if (tid == 0) {
        double u = 0.0, w = 0.0;
        long long c = 0;
        for (int q = 0; q < kTripWaves; ++q) {
            u += s_red[q][0];
            w += s_red[q][1];
            c += s_cnt[q];
        }
        a.ce[2 * base] = u;
        a.ce[2 * base + 1] = w;
        a.cc[base] = c;
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

template <typename T, bool LIST>
static hipError_t launch_triplet_t(hipStream_t st, const TripletArgs &a) {
    const size_t lds = triplet_lds_bytes(a.stage_cap, a.list_cap);
    k_triplet<T, LIST><<<a.ncell, kTripThreads, lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_triplet(hipStream_t st, const TripletArgs &a, bool fp32, bool listing) {
    if (a.ncell <= 0) return hipSuccess;
    if (listing) return fp32 ? launch_triplet_t<float, true>(st, a) : launch_triplet_t<double, true>(st, a);
    return fp32 ? launch_triplet_t<float, false>(st, a) : launch_triplet_t<double, false>(st, a);
}

hipError_t configure_triplet_lds(size_t max_bytes) {
    const void *fns[] = {(const void *)k_triplet<double, false>, (const void *)k_triplet<float, false>,
                         (const void *)k_triplet<double, true>, (const void *)k_triplet<float, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_triplet_gather(hipStream_t st, int64_t n, const double *pf, const int *perm,
                                 double *f, int *flags) {
    if (n > 0) k_triplet_gather<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, pf, perm, f, flags);
    return hipGetLastError();
}

}  // namespace mts
