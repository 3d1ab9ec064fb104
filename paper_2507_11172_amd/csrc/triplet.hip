// Axilrod-Teller-Muto triplet forces (Sec. 2.1) over every triplet whose three pairwise
// distances are all within the three-body cutoff (Sec. 4.1, Fig. 2; Sec. 4.2.2), found
// through linked cells, with Newton's third law applied across each triplet.
//
// The paper's shared-memory traversal (C01, Sec. 4.1) visits every base cell with an
// offset list of cell pairs and cannot use Newton's third law; its conclusion names
// N3-capable traversals as future work.  This kernel is such a traversal, shaped for a
// CDNA wavefront:
//
//  * Ownership.  Particles are ordered by (cell offset, lexicographic in z, y, x; then
//    slot within the cell).  A triplet belongs to its smallest member, the anchor, and
//    its two partners are then "forward" of it: inside the anchor cell after the anchor,
//    or in one of the 13 forward cells of the half stencil.  Every triplet is found once.
//  * One workgroup (one wavefront) per base cell.  The base cell and its 13 forward cells
//    are staged in LDS (FP64 positions plus image-shift codes): the LDS-staged
//    neighbour-cell tile.
//  * Per anchor: the wave filters the tile to the anchor's forward neighbours within
//    rc3 (ballot + prefix count compaction into an LDS list), then sweeps all pairs of
//    that list in a balanced circular order, tests the third edge and evaluates ATM.
//  * Accumulation: the anchor's force stays in registers and is summed across the wave
//    with shuffles; partner forces go to per-tile LDS accumulators (FP64 LDS atomics,
//    one wavefront per tile so the order is fixed).  At the end the tile is flushed to a
//    partial-slot buffer pf[offset][component][particle]; every (offset, particle) slot
//    has exactly one writer, and a gather kernel sums the 14 slots in fixed order.
//    Nothing is accumulated with global float atomics.
//
// Cutoff geometry is FP64 and canonical (the triplet set is bit-identical to the FP64
// oracle's in both precisions); T is the precision of the ATM arithmetic.
#include "common.h"

namespace mts {

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return rsqrtf(x); }

// ATM potential in squared edge lengths a = |u|^2, b = |w|^2, c = |v|^2 (u: anchor->j,
// w: anchor->k, v: j->k).  By the law of cosines the cosine product of Sec. 2.1 is
// t1 t2 t3 / (8abc), t1 = a+b-c, t2 = a-b+c, t3 = b+c-a, so
//   phi = nu [P^-3/2 + 3/8 T P^-5/2],  P = abc,  T = t1 t2 t3.
// Returns phi and g_a = 2 dphi/da, g_b, g_c; the forces are
//   F_anchor = g_a u + g_b w,  F_j = -g_a u + g_c v,  F_k = -g_b w - g_c v.
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
    const T K = T(-1.5) * p32 - T(0.9375) * tt * p52;
    const T Kp = K * ip;              // K / P;  K/a = Kp * b * c
    const T two_nu = T(2) * nu;
    ga = two_nu * fma(Kp, b * c, q * (T(2) * a * t3 - t1 * t2));
    gb = two_nu * fma(Kp, a * c, q * (T(2) * b * t2 - t1 * t3));
    gc = two_nu * fma(Kp, a * b, q * (T(2) * c * t1 - t2 * t3));
    phi = nu * fma(q, tt, p32);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

size_t triplet_lds_bytes(int cap, int lcap) {
    return (size_t)cap * (6 * sizeof(double) + 2 * sizeof(int)) +
           (size_t)lcap * (4 * sizeof(double) + sizeof(int));
}

template <typename T, bool LIST>
__global__ void __launch_bounds__(kWave) k_triplet(TripletArgs a) {
    extern __shared__ double smem[];
    __shared__ int seg_n0;
    const int CAP = a.stage_cap, LC = a.list_cap;
    double *sx = smem, *sy = sx + CAP, *sz = sy + CAP;
    double *ax = sz + CAP, *ay = ax + CAP, *az = ay + CAP;
    double *lux = az + CAP, *luy = lux + LC, *luz = luy + LC, *lua = luz + LC;
    int *scode = (int *)(lua + LC);
    int *sidx = scode + CAP;
    int *lst = sidx + CAP;

    const int base = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const SysDesc &d = a.sd[a.sys_of_cell[base]];
    const int loc = base - d.cell0;
    const int cx = loc % d.nc[0], cy = (loc / d.nc[0]) % d.nc[1], cz = loc / (d.nc[0] * d.nc[1]);
    const double L0 = d.L[0], L1 = d.L[1], L2 = d.L[2];

    // ---- stage the base cell and its 13 forward cells
    int nst = 0;
    for (int o = 0; o < kNumHalf; ++o) {
        int ox, oy, oz, sx_, sy_, sz_;
        half_offset(o, ox, oy, oz);
        const int tx = wrap_cell(cx, ox, d.nc[0], sx_);
        const int ty = wrap_cell(cy, oy, d.nc[1], sy_);
        const int tz = wrap_cell(cz, oz, d.nc[2], sz_);
        const int cell = d.cell0 + (tz * d.nc[1] + ty) * d.nc[0] + tx;
        const int b = a.start[cell], cnt = a.start[cell + 1] - b;
        const int code = (sx_ + 1) | ((sy_ + 1) << 2) | ((sz_ + 1) << 4) | (o << 8);
        for (int t = lane; t < cnt; t += kWave) {
            const int dst = nst + t;
            if (dst < CAP) {
                sx[dst] = a.xs[b + t];
                sy[dst] = a.xs[n + b + t];
                sz[dst] = a.xs[2 * n + b + t];
                scode[dst] = code;
                sidx[dst] = b + t;
            }
        }
        if (o == 0 && lane == 0) seg_n0 = cnt;
        nst += cnt;
    }
    if (nst > CAP) {
        if (lane == 0) atomicOr(a.flags, kFlagStageOverflow);
        nst = CAP;
    }
    for (int t = lane; t < nst; t += kWave) ax[t] = ay[t] = az[t] = 0.0;
    __syncthreads();
    const int nself = min(seg_n0, nst);
    const T nu = (T)a.nu;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));

    double U = 0.0, W = 0.0;
    int cnt_trip = 0;

    for (int ia = 0; ia < nself; ++ia) {
        const double xa = sx[ia], ya = sy[ia], za = sz[ia];  // anchor: base cell, no shift
        // ---- forward neighbours of the anchor within rc3 (stage order > ia)
        int m = 0;
        for (int t0 = ia + 1; t0 < nst; t0 += kWave) {
            const int t = t0 + lane;
            bool in = false;
            double dx = 0, dy = 0, dz = 0, r2 = 0;
            if (t < nst) {
                const int code = scode[t];
                dx = disp1(xa, sx[t], ((code & 3) - 1) * L0);
                dy = disp1(ya, sy[t], (((code >> 2) & 3) - 1) * L1);
                dz = disp1(za, sz[t], (((code >> 4) & 3) - 1) * L2);
                r2 = norm2(dx, dy, dz);
                in = r2 <= a.rc2;
            }
            const uint64_t mask = __ballot(in);
            const int pos = m + __popcll(mask & lt_mask);
            if (in && pos < LC) {
                lst[pos] = t;
                lux[pos] = dx;
                luy[pos] = dy;
                luz[pos] = dz;
                lua[pos] = r2;
            }
            m += __popcll(mask);
        }
        if (m > LC) {
            if (lane == 0) atomicOr(a.flags, kFlagListOverflow);
            m = LC;
        }
        __syncthreads();

        // ---- all pairs (j, k) of the list: circular distance dd = 1 .. m/2, j = 0 .. m-1
        double fax = 0.0, fay = 0.0, faz = 0.0;
        if (m >= 2) {
            const int D = m >> 1;
            const int total = m * D;
            const bool even = (m & 1) == 0;
            const int qstep = kWave / m, rstep = kWave % m;
            int j = lane % m, dd = 1 + lane / m;
            for (int t = lane; t < total; t += kWave) {
                int k = j + dd;
                if (k >= m) k -= m;
                if (!(even && dd == D && j >= D)) {
                    const int tj = lst[j], tk = lst[k];
                    const int cj = scode[tj], ck = scode[tk];
                    const double vx = disp1(sx[tj], sx[tk], ((ck & 3) - (cj & 3)) * L0);
                    const double vy = disp1(sy[tj], sy[tk], (((ck >> 2) & 3) - ((cj >> 2) & 3)) * L1);
                    const double vz = disp1(sz[tj], sz[tk], (((ck >> 4) & 3) - ((cj >> 4) & 3)) * L2);
                    const double c2 = norm2(vx, vy, vz);
                    if (c2 <= a.rc2) {
                        const double ux = lux[j], uy = luy[j], uz = luz[j];
                        const double wx = lux[k], wy = luy[k], wz = luz[k];
                        T phi, ga, gb, gc;
                        atm_terms<T>((T)lua[j], (T)lua[k], (T)c2, nu, phi, ga, gb, gc);
                        const T fix = ga * (T)ux + gb * (T)wx, fiy = ga * (T)uy + gb * (T)wy,
                                fiz = ga * (T)uz + gb * (T)wz;
                        const T fjx = gc * (T)vx - ga * (T)ux, fjy = gc * (T)vy - ga * (T)uy,
                                fjz = gc * (T)vz - ga * (T)uz;
                        const T fkx = -(fix + fjx), fky = -(fiy + fjy), fkz = -(fiz + fjz);
                        fax += (double)fix;
                        fay += (double)fiy;
                        faz += (double)fiz;
                        atomicAdd(&ax[tj], (double)fjx);
                        atomicAdd(&ay[tj], (double)fjy);
                        atomicAdd(&az[tj], (double)fjz);
                        atomicAdd(&ax[tk], (double)fkx);
                        atomicAdd(&ay[tk], (double)fky);
                        atomicAdd(&az[tk], (double)fkz);
                        U += (double)phi;
                        // x . F summed over the triplet, relative to the anchor
                        W += (ux * (double)fjx + uy * (double)fjy + uz * (double)fjz) +
                             (wx * (double)fkx + wy * (double)fky + wz * (double)fkz);
                        ++cnt_trip;
                        if (LIST) {
                            long long slot = (long long)atomicAdd(a.list_n, 1ull);
                            if (slot < a.list_rows) {
                                int p0 = a.perm[sidx[ia]], p1 = a.perm[sidx[tj]], p2 = a.perm[sidx[tk]];
                                int lo = min(p0, min(p1, p2)), hi = max(p0, max(p1, p2));
                                int mid = p0 + p1 + p2 - lo - hi;
                                a.list_ijk[3 * slot] = lo;
                                a.list_ijk[3 * slot + 1] = mid;
                                a.list_ijk[3 * slot + 2] = hi;
                            }
                        }
                    }
                }
                j += rstep;
                dd += qstep;
                if (j >= m) {
                    j -= m;
                    ++dd;
                }
            }
        }
        fax = wave_sum(fax);
        fay = wave_sum(fay);
        faz = wave_sum(faz);
        if (lane == 0) {
            atomicAdd(&ax[ia], fax);
            atomicAdd(&ay[ia], fay);
            atomicAdd(&az[ia], faz);
        }
        __syncthreads();
    }
    __syncthreads();

    // ---- flush the tile's forces: slot (offset, particle) has exactly one writer
    for (int t = lane; t < nst; t += kWave) {
        const int o = scode[t] >> 8;
        const int64_t p = sidx[t];
        a.pf[(3 * o) * n + p] = ax[t];
        a.pf[(3 * o + 1) * n + p] = ay[t];
        a.pf[(3 * o + 2) * n + p] = az[t];
    }
    U = wave_sum(U);
    W = wave_sum(W);
    cnt_trip = wave_sum_int(cnt_trip);
    if (lane == 0) {
        a.ce[2 * base] = U;
        a.ce[2 * base + 1] = W;
        a.cc[base] = cnt_trip;
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
    k_triplet<T, LIST><<<a.ncell, kWave, lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_triplet(hipStream_t st, const TripletArgs &a, bool fp32, bool listing) {
    if (a.ncell <= 0) return hipSuccess;
    if (listing) return fp32 ? launch_triplet_t<float, true>(st, a) : launch_triplet_t<double, true>(st, a);
    return fp32 ? launch_triplet_t<float, false>(st, a) : launch_triplet_t<double, false>(st, a);
}

hipError_t launch_triplet_gather(hipStream_t st, int64_t n, const double *pf, const int *perm,
                                 double *f, int *flags) {
    if (n > 0) k_triplet_gather<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, pf, perm, f, flags);
    return hipGetLastError();
}

}  // namespace mts
