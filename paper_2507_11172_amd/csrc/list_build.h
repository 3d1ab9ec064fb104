// Verlet pair-list build (device code shared by the list-build kernel and the launch
// that runs it next to the triplet kernel): for every particle of a pair-grid cell, the
// sorted indices of all particles within the list radius rc + skin.
#pragma once

#include "common.h"

namespace mts {

constexpr int kListBuildThreads = 4 * kWave;

// ---------------------------------------------------------------- pair list build
// Staged entry: FP32 position relative to the base cell's corner, image shift applied,
// and the sorted particle index.  16 bytes: consecutive lanes read consecutive
// ds_read_b128 words without bank conflicts.
struct alignas(16) BuildEnt {
    float x, y, z;
    int slot;
};

inline size_t list_build_bytes(int cap) { return (size_t)cap * sizeof(BuildEnt); }

// One workgroup of 256 threads builds the list rows of the particles of pair-grid cell
// `base`, staging its 27-cell stencil in `smem` (list_build_bytes(stage_cap) bytes).
__device__ __forceinline__ void list_build_block(const ListBuildArgs &a, int base,
                                                 unsigned char *smem) {
    BuildEnt *tile = (BuildEnt *)smem;
    const int CAP = a.stage_cap;
    const int lane = threadIdx.x;
    const SysDesc &d = a.sd[a.sys_of_cell[base]];
    const int loc = base - d.cell0;
    const int cx = loc % d.nc[0], cy = (loc / d.nc[0]) % d.nc[1], cz = loc / (d.nc[0] * d.nc[1]);
    // positions are staged relative to the base cell's corner: small magnitudes, so
    // FP32 keeps about 1e-7 relative accuracy on every pair distance
    const double ox = cx * (d.L[0] / d.nc[0]), oy = cy * (d.L[1] / d.nc[1]),
                 oz = cz * (d.L[2] / d.nc[2]);

    __shared__ StencilTable<kNumFull> tab;
    int nst = stencil_table<kNumFull, false>(tab, d, cx, cy, cz, a.start);
    int s13 = tab.off[13];
    int nself = tab.off[14] - s13;
    if (a.stats && lane == 0) atomicMax(&a.stats[0], nst);
    if (nst > CAP) {
        if (lane == 0) atomicOr(a.flags, kFlagStageOverflow);
        nst = CAP;
        nself = max(0, min(nself, CAP - s13));
    }
    // workgroup-uniform: the loops below stay scalar
    nst = __builtin_amdgcn_readfirstlane(nst);
    s13 = __builtin_amdgcn_readfirstlane(s13);
    nself = __builtin_amdgcn_readfirstlane(nself);
    for (int t = lane; t < nst; t += kListBuildThreads) {
        const int o = stencil_cell_of<kNumFull>(tab, t);
        const int src = tab.begin[o] + (t - tab.off[o]);
        const int code = tab.code[o];
        const Pos4 ps = a.xs[src];
        BuildEnt e;
        e.x = (float)((ps.x + (double)((code & 3) - 1) * d.L[0]) - ox);
        e.y = (float)((ps.y + (double)(((code >> 2) & 3) - 1) * d.L[1]) - oy);
        e.z = (float)((ps.z + (double)(((code >> 4) & 3) - 1) * d.L[2]) - oz);
        e.slot = src;
        tile[t] = e;
    }
    __syncthreads();

    // the relative margin (1e-5) dwarfs the FP32 rounding of staged positions and of
    // the squared distance (summed with fused multiply-adds), so every pair within the
    // list radius is kept
    const float rv2 = (float)(a.rv2 * (1.0 + 1e-5));
    const int wave = __builtin_amdgcn_readfirstlane(lane / kWave), wl = lane % kWave;
    const int pbase = a.start[base];
    // one wavefront per base-cell particle, all 64 lanes sweeping the tile
    for (int i = wave; i < nself; i += kListBuildThreads / kWave) {
        const int self = s13 + i;
        const BuildEnt pi = tile[self];
        const int64_t p = pbase + i;
        int *row = a.nbr + p * a.nl_cap;
        int cnt = 0;
        for (int t0 = 0; t0 < nst; t0 += kWave) {
            const int t = t0 + wl;
            const bool in = t < nst;
            const BuildEnt e = tile[in ? t : self];
            const float dx = e.x - pi.x, dy = e.y - pi.y, dz = e.z - pi.z;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const bool near = in && t != self && d2 <= rv2;
            // the lane mask from the compares themselves (a ballot of their conjunction
            // would first be materialised in a vector register)
            const uint64_t mask = ballot(in) & ballot(t != self) & ballot(d2 <= rv2);
            const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                      (unsigned)(mask >> 32),
                                      __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            if (near && pos < a.nl_cap) row[pos] = e.slot;
            cnt += __popcll(mask);
        }
        if (wl == 0) {
            a.nn[p] = min(cnt, a.nl_cap);
            if (cnt > a.nl_cap) atomicOr(a.flags, kFlagPairList);
            if (a.stats) atomicMax(&a.stats[1], cnt);
        }
    }
}

}  // namespace mts
