// r-RESPA update (Sec. 4.1, Algorithm 2) and the FP64 energy reductions.
//
// k_int fuses, per particle, every velocity/position update that falls between two force
// evaluations -- the previous step's F2 kick, the F3 half kicks that close one outer cycle
// and open the next, and the drift -- so one launch replaces four.  It is an elementwise
// FP64 stream over x, v and the force caches (HBM-bound) and keeps the exact expression
// order of Algorithm 2:
//   kick2:  v <- v + dt/(2m) * (F2(x^i) + F2(x^{i+1}))
//   kick3:  v <- v + dt*s/(2m) * F3
//   drift:  x <- wrap(x + dt*v + dt^2/(2m) * F2(x^i))
// Reductions sum in a fixed order (per-thread strided sums, then an LDS tree), one
// workgroup per system, so energies are bitwise reproducible.
#include "common.h"

namespace mts {

__global__ void __launch_bounds__(256) k_int(IntArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const SysDesc &d = a.sd[a.sys_of[i]];
    double xn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t q = 3 * i + k;
        double vq = a.v[q];
        if (a.kick2) vq = vq + a.c2 * (a.f2prev[q] + a.f2cur[q]);
        if (a.kick3_end) vq = vq + a.c3 * a.f3[q];
        if (a.kick3_start) vq = vq + a.c3 * a.f3[q];
        a.v[q] = vq;
        if (a.drift) {
            const double xd = a.x[q] + a.dt * vq + a.cx * a.f2cur[q];
            xn[k] = a.open ? xd : wrap1(xd, d.L[k]);
            a.x[q] = xn[k];
        }
    }
    if (!a.drift) return;
    if (a.xs) {
        Pos4 w;
        w.x = xn[0];
        w.y = xn[1];
        w.z = xn[2];
        w.w = 0.0;
        a.xs[a.inv_perm[i]] = w;
    }
    if (a.x_ref) {
        const int64_t ir = 3 * (int64_t)a.inv_perm[i];  // x_ref is in the pair grid's order
        double dd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double t = xn[k] - a.x_ref[ir + k];
            const double h = 0.5 * d.L[k];
            t = t > h ? t - d.L[k] : (t < -h ? t + d.L[k] : t);
            dd[k] = t;
        }
        if (!(norm2(dd[0], dd[1], dd[2]) <= a.half_skin2)) atomicOr(a.flags, kFlagSkin);
    }
}

constexpr int kRed = 256;
constexpr int kRedBatch = 4;  // strides of particles whose loads are in flight together

// Wave-wide sum by butterfly shuffles (fixed order: bitwise reproducible), in every lane.
__device__ __forceinline__ double wave_sum_xor(double v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

// One launch per reduction.  Block (system s, chunk c) sums a fixed contiguous chunk of the
// system's particles (kinetic, pair energy/virial) and cells (triplet energy/virial/count)
// and stores the six partials; the block that finishes a system's chunks last (a
// device-scope counter per system) then sums that system's partials in a fixed order (lane
// l adds chunks l, l + 64, ... in turn, then a butterfly) and writes its record.  A system
// has red_chunks(n) chunks; blocks beyond them (a batch of unequal systems) exit at once.
// The last system to finish advances the record row and every counter is left at zero for
// the next launch, so the kernel can be replayed from a graph.
__global__ void __launch_bounds__(kRed) k_reduce(ReduceArgs a) {
    __shared__ double red[kRed / kWave][6];
    __shared__ int s_last;
    const int s = blockIdx.x / a.chunks, c = blockIdx.x % a.chunks;
    const int t = threadIdx.x;
    const SysDesc &d = a.sd[s];
    const int nch = red_chunks(d.n);
    if (c >= nch) return;
    const int64_t lp = (d.n + nch - 1) / nch;
    const int64_t pb = d.p0 + min(d.n, c * lp), pe = d.p0 + min(d.n, (c + 1) * lp);
    const int lc = (d.ncell + nch - 1) / nch;
    const int cb = d.cell0 + min(d.ncell, c * lc), ce = d.cell0 + min(d.ncell, (c + 1) * lc);
    double v6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // K, U2, U3, W2, W3, count
    // particles in batches of kRedBatch strides: the batch's loads are all issued before
    // its values are added (in the same order as one stride at a time)
    if (a.v)
        for (int64_t i0 = pb + t; i0 < pe; i0 += kRedBatch * kRed) {
            double sq[kRedBatch];
#pragma unroll
            for (int u = 0; u < kRedBatch; ++u) {
                const int64_t i = i0 + (int64_t)u * kRed;
                sq[u] = 0.0;
                if (i < pe) {
                    const double vx = a.v[3 * i], vy = a.v[3 * i + 1], vz = a.v[3 * i + 2];
                    sq[u] = (vx * vx + vy * vy) + vz * vz;
                }
            }
#pragma unroll
            for (int u = 0; u < kRedBatch; ++u)
                if (i0 + (int64_t)u * kRed < pe) v6[0] += sq[u];
        }
    if (a.pe)
        for (int64_t p0 = pb + t; p0 < pe; p0 += kRedBatch * kRed) {
            double2 e[kRedBatch];
#pragma unroll
            for (int u = 0; u < kRedBatch; ++u) {
                const int64_t p = p0 + (int64_t)u * kRed;
                e[u] = p < pe ? reinterpret_cast<const double2 *>(a.pe)[p] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < kRedBatch; ++u)
                if (p0 + (int64_t)u * kRed < pe) {
                    v6[1] += e[u].x;
                    v6[3] += e[u].y;
                }
        }
    if (a.ce)
        for (int q = cb + t; q < ce; q += kRed) {
            v6[2] += a.ce[2 * q];
            v6[4] += a.ce[2 * q + 1];
        }
    if (a.cc)
        for (int q = cb + t; q < ce; q += kRed) v6[5] += (double)a.cc[q];
#pragma unroll
    for (int k = 0; k < 6; ++k) v6[k] = wave_sum_xor(v6[k]);
    if (t % kWave == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k) red[t / kWave][k] = v6[k];
    __syncthreads();
    if (t == 0) {
        double *o = a.part + 6 * ((size_t)s * a.chunks + c);
        for (int k = 0; k < 6; ++k) {
            double r = 0.0;
            for (int w = 0; w < kRed / kWave; ++w) r += red[w][k];
            o[k] = r;
        }
        __threadfence();  // the partials before the count (release)
        s_last = atomicAdd(&a.done[s], 1) == nch - 1;
    }
    __syncthreads();
    if (!s_last || t >= kWave) return;
    __threadfence();  // acquire: every chunk's partials of system s are visible
    static_assert(kRedChunks == kWave, "chunk counts are whole waves");
    const double *part = a.part + 6 * ((size_t)s * a.chunks + t);
    double r[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < nch; q += kWave)
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] += part[6 * q + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k] = wave_sum_xor(r[k]);
    if (t != 0) return;
    a.done[s] = 0;
    const double kin = r[0] * a.half_mass;
    double *out = a.out;
    if (out) {
        if (a.row) out += (int64_t)a.row[0] * a.nsys * a.stride;
        out += (int64_t)s * a.stride;
        if (a.stride == kNE) {
            out[0] = kin; out[1] = r[1]; out[2] = r[2]; out[3] = r[3]; out[4] = r[4];
        } else {
            out[0] = a.pe ? r[1] : r[2];
            out[1] = a.pe ? r[3] : r[4];
        }
    }
    if (a.count_out) a.count_out[s] = (long long)r[5];
    bool ok = true;
    for (int q = 0; q < 5; ++q) ok = ok && isfinite(r[q]);
    if (!ok) atomicOr(a.flags, kFlagNonFinite);
    // the last system advances the row: every system has read it by then
    __threadfence();
    if (atomicAdd(&a.done[a.nsys], 1) == a.nsys - 1) {
        a.done[a.nsys] = 0;
        if (a.row) a.row[0] += 1;
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_int(hipStream_t st, const IntArgs &a) {
    if (a.n > 0) k_int<<<blocks_for(a.n, 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const ReduceArgs &a) {
    if (a.nsys <= 0) return hipSuccess;
    if (a.chunks < kRedChunks || a.chunks > kRedChunksMax || a.chunks % kRedChunks)
        return hipErrorInvalidValue;
    k_reduce<<<a.nsys * a.chunks, kRed, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_set_int(hipStream_t st, int *p, int v) {
    k_set_int<<<1, 1, 0, st>>>(p, v);
    return hipGetLastError();
}


}  // namespace mts
