// Lennard-Jones 12-6 pair forces (Sec. 2.1), evaluated every inner step of r-RESPA
// (Sec. 4.1, Algorithm 2).
//
// GPU formulation: each particle gathers its own force from the full 3x3x3 stencil of
// linked cells, so no force is ever scattered to another particle (no atomics, a fixed
// summation order, bitwise-reproducible results).  Newton's third law is not used for
// pairs: on a GPU it would trade a 2x cheaper arithmetic for a scatter of N x 27 partial
// forces through HBM, which costs more than the pair arithmetic it saves.
//
// G lanes cooperate on one particle, splitting the 27 stencil cells round-robin, and
// combine with a fixed butterfly of cross-lane shuffles.  Cutoff geometry is always FP64
// and canonical (bit-identical pair set in both precisions); T is the precision of the
// LJ arithmetic.  Per-particle forces accumulate in FP64.
#include "common.h"

namespace mts {

template <typename T>
__device__ __forceinline__ void lj_terms(double r2, T sigma2, T eps24, T eps4, T &fr, T &e) {
    const T inv = T(1) / T(r2);
    const T s2 = sigma2 * inv;
    const T s6 = s2 * s2 * s2;
    const T s12 = s6 * s6;
    fr = eps24 * (T(2) * s12 - s6) * inv;  // force on the partner is fr * d
    e = eps4 * (s12 - s6);
}

template <typename T, int G>
__global__ void __launch_bounds__(256) k_pair(PairArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / G;
    const int r = (int)(gid % G);
    const int64_t n = a.n;
    const bool active = p < n;
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
    if (active) {
        const SysDesc &d = a.sd[a.sys_of[p]];
        const double xp = a.xs[p], yp = a.xs[n + p], zp = a.xs[2 * n + p];
        const int cx = cell_coord(xp, d.q[0], d.nc[0]);
        const int cy = cell_coord(yp, d.q[1], d.nc[1]);
        const int cz = cell_coord(zp, d.q[2], d.nc[2]);
        const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
        for (int o = r; o < kNumFull; o += G) {
            int ox, oy, oz, sx, sy, sz;
            full_offset(o, ox, oy, oz);
            const int tx = wrap_cell(cx, ox, d.nc[0], sx);
            const int ty = wrap_cell(cy, oy, d.nc[1], sy);
            const int tz = wrap_cell(cz, oz, d.nc[2], sz);
            const double Sx = sx * d.L[0], Sy = sy * d.L[1], Sz = sz * d.L[2];
            const int cell = d.cell0 + (tz * d.nc[1] + ty) * d.nc[0] + tx;
            const int qb = a.start[cell], qe = a.start[cell + 1];
            for (int q = qb; q < qe; ++q) {
                if (o == 13 && q == p) continue;
                const double dx = disp1(xp, a.xs[q], Sx);
                const double dy = disp1(yp, a.xs[n + q], Sy);
                const double dz = disp1(zp, a.xs[2 * n + q], Sz);
                const double r2 = norm2(dx, dy, dz);
                if (r2 <= a.rc2) {
                    T fr, e;
                    lj_terms<T>(r2, sigma2, eps24, eps4, fr, e);
                    fx -= (double)(fr * (T)dx);
                    fy -= (double)(fr * (T)dy);
                    fz -= (double)(fr * (T)dz);
                    u += (double)e - a.ushift;
                    w += (double)(fr * (T)r2);
                }
            }
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        fx += __shfl_xor(fx, m);
        fy += __shfl_xor(fy, m);
        fz += __shfl_xor(fz, m);
        u += __shfl_xor(u, m);
        w += __shfl_xor(w, m);
    }
    if (active && r == 0) {
        const int64_t i = a.perm[p];
        a.f[3 * i] = fx;
        a.f[3 * i + 1] = fy;
        a.f[3 * i + 2] = fz;
        // every pair is visited from both ends: half of each pair energy and virial
        a.pe[2 * p] = 0.5 * u;
        a.pe[2 * p + 1] = 0.5 * w;
        if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz) || !isfinite(u))
            atomicOr(a.flags, kFlagNonFinite);
    }
}

template <typename T>
static hipError_t launch_pair_t(hipStream_t st, const PairArgs &a, int G) {
    const int64_t threads = a.n * (int64_t)G;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (blocks == 0) return hipSuccess;
    switch (G) {
        case 1: k_pair<T, 1><<<blocks, 256, 0, st>>>(a); break;
        case 2: k_pair<T, 2><<<blocks, 256, 0, st>>>(a); break;
        case 4: k_pair<T, 4><<<blocks, 256, 0, st>>>(a); break;
        case 8: k_pair<T, 8><<<blocks, 256, 0, st>>>(a); break;
        case 16: k_pair<T, 16><<<blocks, 256, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pair(hipStream_t st, const PairArgs &a, bool fp32, int lanes_per_particle) {
    return fp32 ? launch_pair_t<float>(st, a, lanes_per_particle)
                : launch_pair_t<double>(st, a, lanes_per_particle);
}

}  // namespace mts
