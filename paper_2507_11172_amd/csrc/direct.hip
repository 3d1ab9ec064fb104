// DirectSum: every pair and every triplet of a system, with no cutoff and no periodic
// images (the paper's accuracy reference, Sec. 3.1: all interactions of all particles;
// open boundaries, Sec. 4.1 notes that its DirectSum has no boundary conditions).  Same
// LJ and ATM terms as the cutoff path (Sec. 2.1); the triplet set is i < j < k over the
// system, C(N, 3) of them.
//
// k_direct_triplet is the compute-bound kernel: O(N^3) ATM evaluations, Newton's third
// law across each triplet.  Particles form blocks of 64 (one per lane).  A workgroup of
// four waves takes a block triple (I <= J <= K) -- equal work per workgroup, and enough
// workgroups to fill the chip from a few hundred particles on:
//  * lane l owns particle i = 64 I + l; the waves split the j of block J (or of the task's
//    part of it, when a small system's triples are split to fill the chip); for each j the
//    wave sweeps the 64 k of block K in 64 steps, lane l taking k-slot (l + t) mod 64 at
//    step t, so that every lane evaluates one triplet per step with no divergence;
//  * F_i stays in the lane's registers, F_j is summed across the wave once per (j, K),
//    and F_k is accumulated in the register of lane "k-slot": at step t lane m pulls the
//    contribution of lane (m - t) mod 64 by a cross-lane permute -- no atomics;
//  * the partial forces of a task go to its own slots (pI, pJ, pK) and k_direct_gather
//    sums, for each particle, every slot that holds a contribution to it in a fixed
//    order.  Results are bitwise reproducible.
// Block triples with I = J or J = K mask the triplets that are not i < j < k.  Positions
// are FP64; T is the precision of the ATM arithmetic; forces accumulate in FP64.
#include "atm.h"
#include "common.h"

namespace mts {

constexpr int kDirThreads = 4 * kWave;

__device__ __forceinline__ double dwave_sum(double v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

template <typename T, bool ENERGY>
__global__ void __launch_bounds__(kDirThreads) k_direct_triplet(DirectArgs a) {
    __shared__ double sx[3][3][kDirBlock];     // blocks I, J, K: [component][slot]
    __shared__ double red[4][3][kDirBlock];    // per-wave partials of block K, then of I
    __shared__ double sj[3][kDirBlock];        // F_j partials (one writing wave per j)
    __shared__ double se[4][2];
    const DirectTask tk = a.task[blockIdx.x];
    const SysDesc &d = a.sd[tk.sys];
    const int n = (int)d.n;
    const int64_t p0 = d.p0;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int e = tid; e < 3 * 3 * kDirBlock; e += kDirThreads) {
        const int blk = e / (3 * kDirBlock), c = (e / kDirBlock) % 3, slot = e % kDirBlock;
        const int idx = (blk == 0 ? tk.I : (blk == 1 ? tk.J : tk.K)) * kDirBlock + slot;
        sx[blk][c][slot] = idx < n ? a.x[3 * (p0 + idx) + c] : 0.0;
    }
    for (int e = tid; e < 3 * kDirBlock; e += kDirThreads) sj[e / kDirBlock][e % kDirBlock] = 0.0;
    __syncthreads();
    const T nu = (T)a.nu;
    const int i = tk.I * kDirBlock + lane;
    const bool iv = i < n;
    const double xi = sx[0][0][lane], yi = sx[0][1][lane], zi = sx[0][2][lane];
    double fix = 0.0, fiy = 0.0, fiz = 0.0, U = 0.0, W = 0.0;
    {
        const int K = tk.K;
        double kx = 0.0, ky = 0.0, kz = 0.0;  // F of k-slot `lane` of block K
        for (int jj = tk.j0 + wave; jj < tk.j1; jj += 4) {
            const int j = tk.J * kDirBlock + jj;
            if (j >= n) break;  // wave-uniform
            const double xj = sx[1][0][jj], yj = sx[1][1][jj], zj = sx[1][2][jj];
            const double dux = xj - xi, duy = yj - yi, duz = zj - zi;
            const T ux = (T)dux, uy = (T)duy, uz = (T)duz;
            const T aa = fma(uz, uz, fma(uy, uy, ux * ux));
            const bool ij = iv && i < j;
            // over the 64 steps: F_i = (sum g_a) u + sum g_b w, F_j = -(sum g_a) u + sum g_c v
            double sga = 0.0, bwx = 0.0, bwy = 0.0, bwz = 0.0, cvx = 0.0, cvy = 0.0, cvz = 0.0;
            for (int t = 0; t < kDirBlock; ++t) {
                const int ks = (lane + t) & (kDirBlock - 1);
                const int k = K * kDirBlock + ks;
                const bool ok = ij && j < k && k < n;
                const double xk = sx[2][0][ks], yk = sx[2][1][ks], zk = sx[2][2][ks];
                const double dwx = xk - xi, dwy = yk - yi, dwz = zk - zi;
                const double dvx = xk - xj, dvy = yk - yj, dvz = zk - zj;
                const T wx = (T)dwx, wy = (T)dwy, wz = (T)dwz;
                const T vx = (T)dvx, vy = (T)dvy, vz = (T)dvz;
                const T bb = fma(wz, wz, fma(wy, wy, wx * wx));
                const T cc = fma(vz, vz, fma(vy, vy, vx * vx));
                T phi, ga, gb, gc;
                atm_terms<T>(aa, bb, cc, nu, phi, ga, gb, gc);
                // masked triplets (i = j, j = k, padding) may be non-finite: select, never
                // multiply; zero coefficients then zero every force term
                ga = ok ? ga : T(0);
                gb = ok ? gb : T(0);
                gc = ok ? gc : T(0);
                const double dga = (double)ga, dgb = (double)gb, dgc = (double)gc;
                sga += dga;
                bwx = fma(dgb, dwx, bwx); bwy = fma(dgb, dwy, bwy); bwz = fma(dgb, dwz, bwz);
                cvx = fma(dgc, dvx, cvx); cvy = fma(dgc, dvy, cvy); cvz = fma(dgc, dvz, cvz);
                // F_k = -(g_b w + g_c v), summed in the register of lane k-slot
                const T fkx = fma(gb, wx, gc * vx), fky = fma(gb, wy, gc * vy), fkz = fma(gb, wz, gc * vz);
                const int src = (lane - t) & (kDirBlock - 1);
                kx -= (double)__shfl(fkx, src);
                ky -= (double)__shfl(fky, src);
                kz -= (double)__shfl(fkz, src);
                if (ENERGY) {
                    U += ok ? (double)phi : 0.0;
                    W -= (double)fma(aa, ga, fma(bb, gb, cc * gc));
                }
            }
            fix = fma(sga, dux, fix + bwx);
            fiy = fma(sga, duy, fiy + bwy);
            fiz = fma(sga, duz, fiz + bwz);
            double jx = fma(-sga, dux, cvx), jy = fma(-sga, duy, cvy), jz = fma(-sga, duz, cvz);
            jx = dwave_sum(jx);
            jy = dwave_sum(jy);
            jz = dwave_sum(jz);
            if (lane == 0) {
                sj[0][jj] += jx;
                sj[1][jj] += jy;
                sj[2][jj] += jz;
            }
        }
        red[wave][0][lane] = kx;
        red[wave][1][lane] = ky;
        red[wave][2][lane] = kz;
        __syncthreads();
        if (tid < 3 * kDirBlock) {
            const int c = tid / kDirBlock, slot = tid % kDirBlock;
            const double r = ((red[0][c][slot] + red[1][c][slot]) + red[2][c][slot]) + red[3][c][slot];
            a.pK[(int64_t)blockIdx.x * 3 * kDirBlock + tid] = r;
        }
    }
    __syncthreads();
    red[wave][0][lane] = fix;
    red[wave][1][lane] = fiy;
    red[wave][2][lane] = fiz;
    if (ENERGY) {
        U = dwave_sum(U);
        W = dwave_sum(W);
        if (lane == 0) {
            se[wave][0] = U;
            se[wave][1] = W;
        }
    }
    __syncthreads();
    if (tid < 3 * kDirBlock) {
        const int c = tid / kDirBlock, slot = tid % kDirBlock;
        a.pI[(int64_t)blockIdx.x * 3 * kDirBlock + tid] =
            ((red[0][c][slot] + red[1][c][slot]) + red[2][c][slot]) + red[3][c][slot];
        a.pJ[(int64_t)blockIdx.x * 3 * kDirBlock + tid] = sj[c][slot];
    }
    if (ENERGY && tid == 0) {
        a.ce[2 * blockIdx.x] = ((se[0][0] + se[1][0]) + se[2][0]) + se[3][0];
        a.ce[2 * blockIdx.x + 1] = ((se[0][1] + se[1][1]) + se[2][1]) + se[3][1];
    }
}

// F3 of every particle of one 64-particle block (one workgroup per block): the slots that
// hold contributions to it -- tasks (X, J, K) as I, (I, X, K) as J, (I, J, X) as K, each
// triple's split tasks in order, listed in gslot at set-up -- summed in a fixed order:
// wave w takes every kGatherWaves-th slot of that sequence, and the wave sums are added in
// wave order.
constexpr int kGatherWaves = 16;

__global__ void __launch_bounds__(kGatherWaves * kWave) k_direct_gather(DirectArgs a, double *f) {
    __shared__ double red[kGatherWaves][3][kDirBlock];
    const int s = a.blk_sys[blockIdx.x];
    const SysDesc &d = a.sd[s];
    const int n = (int)d.n;
    const int X = (int)blockIdx.x - a.blk0[s];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int64_t beg = a.gslot0[blockIdx.x], end = a.gslot0[blockIdx.x + 1];
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
    for (int64_t q = beg + wave; q < end; q += kGatherWaves) {
        const int e = a.gslot[q];
        const int role = e >> 30;
        const double *slots = role == 0 ? a.pI : (role == 1 ? a.pJ : a.pK);
        const double *src = slots + (int64_t)(e & 0x3fffffff) * 3 * kDirBlock;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += src[c * kDirBlock + lane];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) red[wave][c][lane] = acc[c];
    __syncthreads();
    if (tid < kDirBlock) {
        const int i = X * kDirBlock + tid;
        if (i < n) {
            double o[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
                for (int w = 0; w < kGatherWaves; ++w) t += red[w][c][tid];
                o[c] = t;
            }
            const int64_t p = d.p0 + i;
            f[3 * p] = o[0];
            f[3 * p + 1] = o[1];
            f[3 * p + 2] = o[2];
            if (!isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[2])) atomicOr(a.flags, kFlagNonFinite);
        }
    }
}

// LJ forces of every pair (no cutoff, no images): one wave per particle gathers its own
// force over all others of its system, lane l taking j = l, l + 64, ... (coalesced reads),
// then a butterfly sum in fixed order -- no scatter, bitwise reproducible, and one wave
// per particle fills the chip from a few hundred particles on.  pe receives half of each
// pair's energy and virial.
template <typename T, bool ENERGY>
__global__ void __launch_bounds__(kDirThreads) k_direct_pair(DirectPairArgs a) {
    const int64_t p = ((int64_t)blockIdx.x * kDirThreads + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (p >= a.n) return;  // whole waves
    const SysDesc &d = a.sd[a.sys_of[p]];
    const int n = (int)d.n;
    const int i = (int)(p - d.p0);
    const double xi = a.x[3 * p], yi = a.x[3 * p + 1], zi = a.x[3 * p + 2];
    const T sigma2 = (T)a.sigma2, eps24 = (T)(24.0 * a.eps), eps4 = (T)(4.0 * a.eps);
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, w = 0.0;
    for (int j = lane; j < n; j += kWave) {
        const int64_t q = d.p0 + j;
        const T dx = (T)(a.x[3 * q] - xi), dy = (T)(a.x[3 * q + 1] - yi), dz = (T)(a.x[3 * q + 2] - zi);
        const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const T inv = T(1) / r2;
        const T s2 = sigma2 * inv;
        const T s6 = s2 * s2 * s2;
        const T s12 = s6 * s6;
        const T fr = eps24 * fma(T(2), s12, -s6) * inv;
        const bool ok = j != i;  // the particle itself (r2 = 0) is selected away
        fx -= ok ? (double)(fr * dx) : 0.0;
        fy -= ok ? (double)(fr * dy) : 0.0;
        fz -= ok ? (double)(fr * dz) : 0.0;
        if (ENERGY) {
            u += ok ? (double)(eps4 * (s12 - s6)) : 0.0;
            w += ok ? (double)(fr * r2) : 0.0;
        }
    }
    fx = dwave_sum(fx);
    fy = dwave_sum(fy);
    fz = dwave_sum(fz);
    if (ENERGY) {
        u = dwave_sum(u);
        w = dwave_sum(w);
    }
    if (lane != 0) return;
    a.f[3 * p] = fx;
    a.f[3 * p + 1] = fy;
    a.f[3 * p + 2] = fz;
    if (ENERGY) {
        a.pe[2 * p] = 0.5 * u;
        a.pe[2 * p + 1] = 0.5 * w;
    }
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz)) atomicOr(a.flags, kFlagNonFinite);
}

hipError_t launch_direct_triplet(hipStream_t st, const DirectArgs &a, bool fp32, bool energy) {
    if (a.ntask <= 0) return hipSuccess;
    if (fp32) {
        if (energy) k_direct_triplet<float, true><<<a.ntask, kDirThreads, 0, st>>>(a);
        else k_direct_triplet<float, false><<<a.ntask, kDirThreads, 0, st>>>(a);
    } else {
        if (energy) k_direct_triplet<double, true><<<a.ntask, kDirThreads, 0, st>>>(a);
        else k_direct_triplet<double, false><<<a.ntask, kDirThreads, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_direct_gather(hipStream_t st, const DirectArgs &a, double *f) {
    if (a.nblk > 0) k_direct_gather<<<a.nblk, kGatherWaves * kWave, 0, st>>>(a, f);
    return hipGetLastError();
}

hipError_t launch_direct_pair(hipStream_t st, const DirectPairArgs &a) {
    if (a.n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.n * kWave + kDirThreads - 1) / kDirThreads);
    if (a.pe != nullptr) k_direct_pair<double, true><<<blocks, kDirThreads, 0, st>>>(a);
    else k_direct_pair<double, false><<<blocks, kDirThreads, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace mts
