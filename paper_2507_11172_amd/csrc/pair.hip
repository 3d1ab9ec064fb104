// Lennard-Jones 12-6 pair forces (Sec. 2.1), evaluated every inner step of r-RESPA
// (Sec. 4.1, Algorithm 2).
//
// GPU formulation: each particle gathers its own force from its neighbours, so no force
// is ever scattered to another particle (no atomics, a fixed summation order,
// bitwise-reproducible results).  Newton's third law is not used for pairs: on a GPU it
// would trade 2x cheaper arithmetic for a scatter of partial forces through memory,
// which costs more than the pair arithmetic it saves.
//
// Three kernels:
//  * k_pair: linked-cell tile kernel.  One workgroup (4 wavefronts) per base cell stages
//    the 27 cells of its stencil in LDS once (FP64 positions + image shifts); groups of
//    16 lanes each take one particle of the base cell and sweep the tile with stride 16.
//    Used for standalone force calls and when no pair list is kept.
//  * k_list_build: the same stencil on the pair-list grid (cells >= rc + skin), one
//    wavefront per particle, FP32 distance test, ballot compaction of every neighbour
//    within rc + skin into the particle's row of the Verlet list.  Runs once per outer
//    r-RESPA cycle.
//  * k_pair_list: 4, 8 or 16 lanes per particle (a tuning choice) walk its list row (four
//    gathers in flight per lane), a DPP butterfly inside the group combines them in
//    fixed order, and
//    the particle's r-RESPA update is fused behind the force (one launch per inner
//    step).  Energies and virials are summed only when asked for (full steps).
// Cutoff geometry is always FP64 and canonical (bit-identical pair set in both
// precisions).  The LJ arithmetic is FP64 in both forms of the library: FP32 issues at the
// FP64 rate here (no packed FP32), and in dense systems FP32 LJ exceeds an energy error of
// 1e-7 per particle (s^12 - s^6 cancels for the many pairs near r = sigma).  The kernels
// keep the arithmetic type T as a template parameter.  Forces accumulate in FP64.
#include "common.h"
#include "list_build.h"

namespace mts {

constexpr int kPairGroup = 16;
constexpr int kPairThreads = 4 * kWave;
constexpr int kPairGroups = kPairThreads / kPairGroup;


// 1/x: hardware estimate refined by two Newton-Raphson steps y <- y (2 - x y).
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

template <typename T>
__device__ __forceinline__ T rcp_t(T x);
template <>
__device__ __forceinline__ double rcp_t<double>(double x) { return rcp_nr(x); }
template <>
__device__ __forceinline__ float rcp_t<float>(float x) { return 1.0f / x; }

template <typename T>
__device__ __forceinline__ void lj_terms(double r2, T sigma2, T eps24, T eps4, T &fr, T &e) {
    const T inv = rcp_t<T>(T(r2));
    const T s2 = sigma2 * inv;
    const T s6 = s2 * s2 * s2;
    const T s12 = s6 * s6;
    fr = eps24 * fma(T(2), s12, -s6) * inv;  // force on the partner is fr * d
    e = eps4 * (s12 - s6);
}

// Tile entry in LDS: FP64 wrapped position and the image shift of the entry (0 or +-L per
// component).  48 bytes, an odd multiple of 16, so that three ds_read_b128 by
// consecutive lanes are free of bank conflicts.
struct alignas(16) PairEnt {
    double x, y, z, sx, sy, sz;
};
static_assert(sizeof(PairEnt) == 48, "48-byte LDS entries");

size_t pair_lds_bytes(int cap) { return (size_t)cap * sizeof(PairEnt); }

template <typename T>
__global__ void __launch_bounds__(kPairThreads) k_pair(PairArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int CAP = a.stage_cap;
    PairEnt *tile = (PairEnt *)smem_raw;
    const int base = blockIdx.x;
    const int lane = threadIdx.x;  // thread index in the workgroup
    const SysDesc &d = a.sd[a.sys_of_cell[base]];
    const int loc = base - d.cell0;
    const int cx = loc % d.nc[0], cy = (loc / d.nc[0]) % d.nc[1], cz = loc / (d.nc[0] * d.nc[1]);

    __shared__ StencilTable<kNumFull> tab;
    int nst = stencil_table<kNumFull, false>(tab, d, cx, cy, cz, a.start);
    const int s13 = tab.off[13];
    int nself = tab.off[14] - s13;
    if (nst > CAP) {
        if (lane == 0) atomicOr(a.flags, kFlagStageOverflow);
        nst = CAP;
        nself = max(0, min(nself, CAP - s13));
    }
    for (int t = lane; t < nst; t += kPairThreads) {
        const int o = stencil_cell_of<kNumFull>(tab, t);
        const int src = tab.begin[o] + (t - tab.off[o]);
        const int code = tab.code[o];
        const Pos4 ps = a.xs[src];
        PairEnt e;
        e.x = ps.x;
        e.y = ps.y;
        e.z = ps.z;
        e.sx = (double)((code & 3) - 1) * d.L[0];
        e.sy = (double)(((code >> 2) & 3) - 1) * d.L[1];
        e.sz = (double)(((code >> 4) & 3) - 1) * d.L[2];
        tile[t] = e;
    }
    __syncthreads();

    const int g = lane / kPairGroup, r = lane % kPairGroup;  // group and lane in group
    const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
    const int pbase = a.start[base];
    for (int ib = 0; ib < nself; ib += kPairGroups) {
        const int i = ib + g;
        const bool act = i < nself;
        const int self = s13 + (act ? i : 0);
        const PairEnt pi = tile[self];
        const int64_t p = pbase + i;
        double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
        for (int t0 = 0; t0 < nst; t0 += kPairGroup) {
            const int t = t0 + r;
            if (act && t < nst && t != self) {
                const PairEnt e = tile[t];
                const double dx = disp1(pi.x, e.x, e.sx);
                const double dy = disp1(pi.y, e.y, e.sy);
                const double dz = disp1(pi.z, e.z, e.sz);
                const double r2 = norm2(dx, dy, dz);
                if (r2 <= a.rc2) {
                    T fr, e4;
                    lj_terms<T>(r2, sigma2, eps24, eps4, fr, e4);
                    fx -= (double)(fr * (T)dx);
                    fy -= (double)(fr * (T)dy);
                    fz -= (double)(fr * (T)dz);
                    u += (double)e4 - a.ushift;
                    w += (double)(fr * (T)r2);
                }
            }
        }
#pragma unroll
        for (int m = 1; m < kPairGroup; m <<= 1) {
            fx += __shfl_xor(fx, m);
            fy += __shfl_xor(fy, m);
            fz += __shfl_xor(fz, m);
            u += __shfl_xor(u, m);
            w += __shfl_xor(w, m);
        }
        if (act && r == 0) {
            const int64_t q = a.perm[p];
            a.f[3 * q] = fx;
            a.f[3 * q + 1] = fy;
            a.f[3 * q + 2] = fz;
            // every pair is visited from both ends: half of each pair energy and virial
            a.pe[2 * p] = 0.5 * u;
            a.pe[2 * p + 1] = 0.5 * w;
            if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz) || !isfinite(u))
                atomicOr(a.flags, kFlagNonFinite);
        }
    }
}

size_t list_build_lds_bytes(int cap) { return list_build_bytes(cap); }

__global__ void __launch_bounds__(kListBuildThreads) k_list_build(ListBuildArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    list_build_block(a, blockIdx.x, smem_raw);
}

hipError_t launch_list_build(hipStream_t st, const ListBuildArgs &a) {
    if (a.ncell <= 0) return hipSuccess;
    k_list_build<<<a.ncell, kPairThreads, list_build_lds_bytes(a.stage_cap), st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- list forces + update

template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over G = 4, 8 or 16 consecutive lanes (inside one DPP row); every lane of the group
// ends with the same value.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 4 || G == 8 || G == 16, "groups of 4, 8 or 16 lanes");
    v += dpp_row<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_row<0x4E>(v);   // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_row<0x141>(v);  // row_half_mirror
    if (G == 16) v += dpp_row<0x140>(v);  // row_mirror
    return v;
}

template <typename T, bool ENERGY>
__device__ __forceinline__ void lj_accumulate(const Pos4 &pi, const Pos4 &e, const double *L,
                                              const double *iL, double rc2, T sigma2, T eps24,
                                              T eps4, double ushift, double &fx, double &fy,
                                              double &fz, double &u, double &w) {
    // minimum image fl(fl(x_q - x_p) + S), S = -L rint((x_q - x_p) / L) in {-L, 0, +L}:
    // the product L * rint(.) is exact, so the fma rounds once, like the addition
    double dx = e.x - pi.x, dy = e.y - pi.y, dz = e.z - pi.z;
    dx = fma(-L[0], rint(dx * iL[0]), dx);
    dy = fma(-L[1], rint(dy * iL[1]), dy);
    dz = fma(-L[2], rint(dz * iL[2]), dz);
    const double r2 = norm2(dx, dy, dz);
    if (r2 <= rc2) {
        T fr, e4;
        lj_terms<T>(r2, sigma2, eps24, eps4, fr, e4);
        fx -= (double)(fr * (T)dx);
        fy -= (double)(fr * (T)dy);
        fz -= (double)(fr * (T)dz);
        if (ENERGY) {
            u += (double)e4 - ushift;
            w += (double)(fr * (T)r2);
        }
    }
}

// Entries per lane per pass: all their index loads, then all their position gathers,
// are in flight together.
constexpr int kListUnroll = 4;

template <typename T, bool ENERGY, int G>
__global__ void __launch_bounds__(256) k_pair_list(PairListArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / G;
    const int r = (int)(gid % G);
    const bool act = p < a.n;

    // The first 64 list entries of the row are loaded before the row length is known
    // (the row is allocated to nl_cap entries; entries past the length are ignored), so
    // that the index loads, the per-particle loads and, next, the operands of the fused
    // update overlap with the position gathers (lane r < 3 owns component r of the
    // update).
    const int64_t pp = act ? p : 0;
    const int *row = a.nbr + pp * a.nl_cap;
    constexpr int U = 64 / G;  // entries per lane in the first pass
    int qn[U];
#pragma unroll
    for (int k = 0; k < U; ++k) qn[k] = row[min(r + k * G, a.nl_cap - 1)];
    const int cnt = act ? a.nn[pp] : 0;
    const Pos4 pi = a.xs[pp];
    const int64_t q = 3 * (int64_t)a.perm[pp] + (r < 3 ? r : 0);  // input order
    const int64_t qs = 3 * pp + (r < 3 ? r : 0);                    // sorted order
    const int64_t qi = a.in_sorted ? qs : q, qo = a.out_sorted ? qs : q;
    const SysDesc &d = a.sd[a.sys_of[pp]];
    const double L[3] = {d.L[0], d.L[1], d.L[2]};
    const double iL[3] = {d.iL[0], d.iL[1], d.iL[2]};
    const bool upd = act && r < 3 && a.v_in != nullptr;
    double vq = 0.0, f2p = 0.0, f3q = 0.0, xq = 0.0, xr = 0.0;
    if (act && r < 3 && a.pf) {
        // F3 of this particle from the 14 partial slots, in slot order
        const int64_t pt = a.inv_perm3[a.perm[pp]];
        const int64_t n = a.n;
        double s3 = 0.0;
#pragma unroll
        for (int o = 0; o < kNumHalf; ++o) s3 += a.pf[(3 * o + r) * n + pt];
        f3q = s3;
        a.f3_out[q] = s3;
        if (!isfinite(s3)) atomicOr(a.flags, kFlagNonFinite);
    }
    if (upd) {
        vq = a.v_in[qi];
        if (a.kick2) f2p = a.f2prev[qi];
        if (!a.pf && (a.kick3_end || a.kick3_start)) f3q = a.f3[q];
        if (a.drift) {
            xq = r == 0 ? pi.x : (r == 1 ? pi.y : pi.z);  // x^i
            if (a.x_ref) xr = a.x_ref[qs];
        }
        if (a.open_next) {
            xq = a.x[q];  // x^k as the caller keeps it
            xr = a.x_ref[qs];
        }
    }

    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
    {
        const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
        {
            Pos4 e[U];
#pragma unroll
            for (int k = 0; k < U; ++k) e[k] = a.xs[r + k * G < cnt ? qn[k] : (int)pp];
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (r + k * G < cnt)
                    lj_accumulate<T, ENERGY>(pi, e[k], L, iL, a.rc2, sigma2, eps24, eps4, a.ushift,
                                             fx, fy, fz, u, w);
        }
        for (int s0 = r + 64; s0 < cnt; s0 += kListUnroll * G) {  // rows longer than 64
            int qn[kListUnroll];
#pragma unroll
            for (int k = 0; k < kListUnroll; ++k) {
                const int s = s0 + k * G;
                qn[k] = s < cnt ? row[s] : (int)pp;
            }
            Pos4 e[kListUnroll];
#pragma unroll
            for (int k = 0; k < kListUnroll; ++k) e[k] = a.xs[qn[k]];
#pragma unroll
            for (int k = 0; k < kListUnroll; ++k)
                if (s0 + k * G < cnt)
                    lj_accumulate<T, ENERGY>(pi, e[k], L, iL, a.rc2, sigma2, eps24, eps4, a.ushift,
                                             fx, fy, fz, u, w);
        }
    }
    fx = group_sum<G>(fx);
    fy = group_sum<G>(fy);
    fz = group_sum<G>(fz);
    if (ENERGY) {
        u = group_sum<G>(u);
        w = group_sum<G>(w);
    }

    // ---- fused update of component r, in Algorithm 2's order
    double dd2 = 0.0;
    if (act && r < 3) {
        const double F = r == 0 ? fx : (r == 1 ? fy : fz);
        a.f[qo] = F;
        if (upd) {
            if (a.kick2) vq = vq + a.c2 * (f2p + F);
            if (a.kick3_end) vq = vq + a.c3 * f3q;
            if (a.kick3_start) vq = vq + a.c3 * f3q;
            a.v_out[qo] = vq;
            if (a.drift) {
                const double Lr = L[r];
                const double xn = wrap1(xq + a.dt * vq + a.cx * F, Lr);
                if (a.x) a.x[q] = xn;
                if (a.xs_out) reinterpret_cast<double *>(a.xs_out + p)[r] = xn;
                if (a.x_ref) {
                    double t = xn - xr;
                    const double h = 0.5 * Lr;
                    t = t > h ? t - Lr : (t < -h ? t + Lr : t);
                    dd2 = t * t;
                }
            }
            if (a.open_next) {  // the next cycle's F3 half kick and first drift
                const double vn = vq + a.c3 * f3q;
                a.v_next[qs] = vn;
                a.f2_next[qs] = F;
                const double Lr = L[r];
                const double xn = wrap1(xq + a.dt * vn + a.cx * F, Lr);
                reinterpret_cast<double *>(a.xs_next + p)[r] = xn;
                double t = xn - xr;
                const double h = 0.5 * Lr;
                t = t > h ? t - Lr : (t < -h ? t + Lr : t);
                dd2 = t * t;
            }
        }
    }
    // displacement since the list build: (dx^2 + dy^2) + dz^2 in lane r = 0
    const double d1 = __shfl_down(dd2, 1, G);
    const double d2 = __shfl_down(dd2, 2, G);
    if (act && r == 0) {
        if (ENERGY) {
            a.pe[2 * p] = 0.5 * u;
            a.pe[2 * p + 1] = 0.5 * w;
        }
        if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz) || (ENERGY && !isfinite(u)))
            atomicOr(a.flags, kFlagNonFinite);
        if (upd && ((a.drift && a.x_ref) || a.open_next) && !((dd2 + d1) + d2 <= a.half_skin2))
            atomicOr(a.flags, kFlagSkin);
    }
}

template <int G>
static hipError_t launch_pair_list_g(hipStream_t st, const PairListArgs &a) {
    const int64_t threads = a.n * G;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (a.pe != nullptr) k_pair_list<double, true, G><<<blocks, 256, 0, st>>>(a);
    else k_pair_list<double, false, G><<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_pair_list(hipStream_t st, const PairListArgs &a) {
    if (a.lanes == 4) return launch_pair_list_g<4>(st, a);
    if (a.lanes == 8) return launch_pair_list_g<8>(st, a);
    if (a.lanes == 16) return launch_pair_list_g<16>(st, a);
    return hipErrorInvalidValue;
}

hipError_t configure_triplet_lds(size_t max_bytes);

hipError_t configure_kernel_lds(size_t max_bytes) {
    const void *fns[] = {(const void *)k_pair<double>, (const void *)k_list_build};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
        if (e != hipSuccess) return e;
    }
    return configure_triplet_lds(max_bytes);
}

hipError_t launch_pair(hipStream_t st, const PairArgs &a) {
    if (a.ncell <= 0) return hipSuccess;
    const size_t lds = pair_lds_bytes(a.stage_cap);
    k_pair<double><<<a.ncell, kPairThreads, lds, st>>>(a);
    return hipGetLastError();
}

}  // namespace mts
