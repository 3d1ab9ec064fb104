// Lennard-Jones 12-6 pair forces (Sec. 2.1), evaluated every inner step of r-RESPA
// (Sec. 4.1, Algorithm 2).
//
// GPU formulation: each particle gathers its own force from the full 3x3x3 stencil of
// linked cells, so no force is ever scattered to another particle (no atomics, a fixed
// summation order, bitwise-reproducible results).  Newton's third law is not used for
// pairs: on a GPU it would trade 2x cheaper arithmetic for a scatter of N x 27 partial
// forces through HBM, which costs more than the pair arithmetic it saves.
//
// One workgroup (4 wavefronts) per base cell stages the 27 cells of its stencil in LDS
// once (FP64 positions + image-shift code).  Groups of 16 lanes each take one particle
// of the base cell and sweep the tile with stride 16; a 4-step shuffle butterfly
// combines the group.
// Cutoff geometry is always FP64 and canonical (bit-identical pair set in both
// precisions); T is the precision of the LJ arithmetic.  Forces accumulate in FP64.
#include "common.h"

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

size_t pair_lds_bytes(int cap) { return (size_t)cap * (sizeof(PairEnt) + sizeof(int)); }

template <typename T>
__global__ void __launch_bounds__(kPairThreads) k_pair(PairArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int CAP = a.stage_cap;
    PairEnt *tile = (PairEnt *)smem_raw;
    int *tslot = (int *)(tile + CAP);  // sorted index of each tile entry
    const int base = blockIdx.x;
    const int lane = threadIdx.x;  // thread index in the workgroup
    const int64_t n = a.n;
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
        PairEnt e;
        e.x = a.xs[src];
        e.y = a.xs[n + src];
        e.z = a.xs[2 * n + src];
        e.sx = (double)((code & 3) - 1) * d.L[0];
        e.sy = (double)(((code >> 2) & 3) - 1) * d.L[1];
        e.sz = (double)(((code >> 4) & 3) - 1) * d.L[2];
        tile[t] = e;
        tslot[t] = src;
    }
    __syncthreads();

    const int g = lane / kPairGroup, r = lane % kPairGroup;  // group and lane in group
    const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
    const int pbase = a.start[base];
    const bool build = a.nbr != nullptr;
    const int gshift = kPairGroup * ((lane % kWave) / kPairGroup);  // group's bits in the ballot
    for (int ib = 0; ib < nself; ib += kPairGroups) {
        const int i = ib + g;
        const bool act = i < nself;
        const int self = s13 + (act ? i : 0);
        const PairEnt pi = tile[self];
        const int64_t p = pbase + i;
        double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
        int cnt = 0;  // pair-list entries of this group's particle (uniform in the group)
        for (int t0 = 0; t0 < nst; t0 += kPairGroup) {
            const int t = t0 + r;
            bool near = false;
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
                near = r2 <= a.rcv2;
            }
            if (build) {
                const uint64_t mask = __ballot(near);
                const unsigned gbits = (unsigned)(mask >> gshift) & 0xffffu;
                const int pos = cnt + __popc(gbits & ((1u << r) - 1u));
                if (near && pos < a.nl_cap) a.nbr[p * a.nl_cap + pos] = tslot[t];
                cnt += __popc(gbits);
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
            if (build) {
                a.nn[p] = min(cnt, a.nl_cap);
                if (cnt > a.nl_cap) atomicOr(a.flags, kFlagPairList);
            }
        }
    }
}

// Per-step pair forces from the list: 8 lanes per particle take every 8th list entry,
// and a DPP butterfly inside each 8-lane row segment combines them in fixed order.
constexpr int kListGroup = 8;

template <int CTRL>
__device__ __forceinline__ double dpp8(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double sum8(double v) {
    v += dpp8<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp8<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp8<0x141>(v);  // row_half_mirror: lane i <- lane 7-i within 8
    return v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_pair_list(PairListArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / kListGroup;
    const int r = (int)(gid % kListGroup);
    const bool act = p < a.n;
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
    if (act) {
        const int64_t n = a.n;
        const SysDesc &d = a.sd[a.sys_of[p]];
        const double L0 = d.L[0], L1 = d.L[1], L2 = d.L[2];
        const double h0 = 0.5 * L0, h1 = 0.5 * L1, h2 = 0.5 * L2;
        const double xp = a.xs[p], yp = a.xs[n + p], zp = a.xs[2 * n + p];
        const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
        const int cnt = a.nn[p];
        const int *row = a.nbr + p * a.nl_cap;
        for (int s = r; s < cnt; s += kListGroup) {
            const int64_t q = row[s];
            // minimum image by comparison: fl(fl(x_q - x_p) + S), S in {-L, 0, +L}
            double dx = a.xs[q] - xp, dy = a.xs[n + q] - yp, dz = a.xs[2 * n + q] - zp;
            dx = dx > h0 ? dx - L0 : (dx < -h0 ? dx + L0 : dx);
            dy = dy > h1 ? dy - L1 : (dy < -h1 ? dy + L1 : dy);
            dz = dz > h2 ? dz - L2 : (dz < -h2 ? dz + L2 : dz);
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
    fx = sum8(fx);
    fy = sum8(fy);
    fz = sum8(fz);
    u = sum8(u);
    w = sum8(w);
    if (act && r == 0) {
        const int64_t q = a.perm[p];
        a.f[3 * q] = fx;
        a.f[3 * q + 1] = fy;
        a.f[3 * q + 2] = fz;
        a.pe[2 * p] = 0.5 * u;
        a.pe[2 * p + 1] = 0.5 * w;
        if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz) || !isfinite(u))
            atomicOr(a.flags, kFlagNonFinite);
    }
}

hipError_t launch_pair_list(hipStream_t st, const PairListArgs &a, bool fp32) {
    const int64_t threads = a.n * kListGroup;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (fp32)
        k_pair_list<float><<<blocks, 256, 0, st>>>(a);
    else
        k_pair_list<double><<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t configure_triplet_lds(size_t max_bytes);

hipError_t configure_kernel_lds(size_t max_bytes) {
    const void *fns[] = {(const void *)k_pair<double>, (const void *)k_pair<float>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
        if (e != hipSuccess) return e;
    }
    return configure_triplet_lds(max_bytes);
}

hipError_t launch_pair(hipStream_t st, const PairArgs &a, bool fp32) {
    if (a.ncell <= 0) return hipSuccess;
    const size_t lds = pair_lds_bytes(a.stage_cap);
    if (fp32)
        k_pair<float><<<a.ncell, kPairThreads, lds, st>>>(a);
    else
        k_pair<double><<<a.ncell, kPairThreads, lds, st>>>(a);
    return hipGetLastError();
}

}  // namespace mts
