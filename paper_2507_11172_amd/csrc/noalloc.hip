// Triplet forces of one periodic system without a handle and without allocating device
// memory: the cell grid, the tile capacities' bookkeeping, the partial-force slots and
// the counters live in one file-scope device array (`scratch`), which every GPU the
// library runs on holds until the process ends.  The kernels are the handle path's own
// (binning, triplet tiles, slot gather, energy reduction); only the buffers differ.
//
// Host code never passes `scratch` itself to a kernel: in host code that name is a
// stand-in, not a device address.  The device address of each GPU's copy is looked up
// once per device with hipGetSymbolAddress and kept in g_scratch[device].
#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/mts.h"
#include "common.h"

using namespace mts;

static __device__ __align__(256) unsigned char scratch[MTS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};  // device address of each GPU's scratch
size_t g_max_lds[kMaxDevices] = {};          // dynamic LDS a workgroup may use

__global__ void k_fill_int(int *p, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_put_desc(SysDesc *dst, SysDesc d) { *dst = d; }

hipError_t fill_int(hipStream_t st, int *p, int64_t n, int v) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    k_fill_int<<<blocks, 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

// Carves [bytes] from the scratch block at 256-byte alignment.
struct Carver {
    unsigned char *base;
    size_t used = 0;
    template <typename T>
    T *take(size_t count) {
        T *p = (T *)(base + used);
        used += (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
        return p;
    }
};

// Once per device, with that device current: the scratch address and the kernels' LDS limit.
mts_status device_setup(int dev, unsigned char **ptr, size_t *max_lds) {
    if (dev < 0 || dev >= kMaxDevices) return MTS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return MTS_ERR_HIP;
        }
        int lds = 0;
        size_t m = 64 * 1024;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            m = (size_t)lds;
        m = m > kStaticLdsReserve ? m - kStaticLdsReserve : m;  // room for the static LDS
        if (configure_kernel_lds(m) != hipSuccess) m = 64 * 1024 - kStaticLdsReserve;
        (void)hipGetLastError();
        g_scratch[dev] = (unsigned char *)p;
        g_max_lds[dev] = m;
    }
    *ptr = g_scratch[dev];
    *max_lds = g_max_lds[dev];
    return MTS_OK;
}

}  // namespace

extern "C" mts_status mts_compute_triplet_forces_static(const mts_params *params, int64_t n,
                                                        const double box[3], const double *x,
                                                        double *f3, double *ew, void *stream) {
    if (!params || !box || n < 0 || ((!x || !f3) && n > 0)) return MTS_ERR_INVALID_ARG;
    if (params->method != MTS_CUTOFF || params->k_outer > 1) return MTS_ERR_UNSUPPORTED;
    if (params->precision != MTS_FP64 && params->precision != MTS_FP32) return MTS_ERR_INVALID_ARG;
    const double rc3 = params->rc_triplet;
    if (!(rc3 > 0.0) || !std::isfinite(rc3) || !std::isfinite(params->nu)) return MTS_ERR_INVALID_ARG;
    if (n >= (int64_t)1 << 30) return MTS_ERR_UNSUPPORTED;
    const double margin = 1.0 + 1e-9;  // cells strictly wider than the cutoff, as on handles
    SysDesc d{};
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        const double L = box[k];
        if (!(L > 0.0) || !std::isfinite(L)) return MTS_ERR_INVALID_ARG;
        if (!(L > 2.0 * std::max(rc3, params->rc_pair) * margin)) return MTS_ERR_BOX_TOO_SMALL;
        d.L[k] = L;
        d.iL[k] = 1.0 / L;
        d.nc[k] = (int)std::floor(L / (rc3 * margin));
        if (d.nc[k] < 2) return MTS_ERR_BOX_TOO_SMALL;
        d.q[k] = (double)d.nc[k] / L;
        ncell *= d.nc[k];
    }
    if (ncell >= (int64_t)1 << 30) return MTS_ERR_UNSUPPORTED;
    d.ncell = (int)ncell;
    d.whole = ncell < kNumHalf ? 1 : 0;  // as on handles: tiny boxes are staged whole
    d.cell0 = 0;
    d.p0 = 0;
    d.n = n;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MTS_ERR_HIP;
    unsigned char *base = nullptr;
    size_t max_lds = 0;
    mts_status r = device_setup(dev, &base, &max_lds);
    if (r != MTS_OK) return r;

    // capacities: the handle's default heuristics (a cell of volume h^3 holds about
    // rho h^3 particles at rho = max(0.9, 1.2 x the mean density); a forward list about
    // half a cutoff sphere, sized for a whole one at 1.25 x that density)
    const bool fp32 = params->precision == MTS_FP32;
    const double vol = d.L[0] * d.L[1] * d.L[2];
    const double rho = std::max(0.9, 1.2 * (double)n / vol);
    const double vcell = rho * (d.L[0] / d.nc[0]) * (d.L[1] / d.nc[1]) * (d.L[2] / d.nc[2]);
    const int list_cap = std::min(256, ((int)std::ceil(1.25 * rho * (4.0 / 3.0) * M_PI * rc3 * rc3 * rc3) + 8 + 15) / 16 * 16);
    int stage_cap = d.whole ? ((int)n + 31) / 32 * 32
                            : ((int)std::ceil(kNumHalf * vcell * 1.1) + 16 + 31) / 32 * 32;
    while (stage_cap > 32 && triplet_lds_bytes(stage_cap, list_cap, fp32) > max_lds) stage_cap -= 32;
    if (triplet_lds_bytes(stage_cap, list_cap, fp32) > max_lds) return MTS_ERR_UNSUPPORTED;

    // the scratch layout of this call
    const int ntile = (int)((ncell + kScanTile - 1) / kScanTile);
    Carver cv{base};
    SysDesc *sd = cv.take<SysDesc>(1);
    int *flags = cv.take<int>(1);
    int *tile_obs = cv.take<int>(1);
    int *red_done = cv.take<int>(2);
    int *count = cv.take<int>(ncell);
    int *start = cv.take<int>(ncell + 1);
    int *start_loc = cv.take<int>(ncell);
    int *tile_sum = cv.take<int>(2 * (size_t)ntile + 1);
    int *sys_of_cell = cv.take<int>(ncell);
    int *sys_of = cv.take<int>(n);
    int *cell_of = cv.take<int>(n);
    int *rank = cv.take<int>(n);
    int *tmp = cv.take<int>(n);
    int *perm = cv.take<int>(n);
    int *inv_perm = cv.take<int>(n);
    Pos4 *xs = cv.take<Pos4>(n);
    double *pf = cv.take<double>((size_t)kNumHalf * 3 * n);
    double *ce = cv.take<double>(2 * (size_t)ncell);
    double *part = cv.take<double>((size_t)red_chunks(n) * 6);
    if (cv.used > (size_t)MTS_STATIC_SCRATCH_BYTES) return MTS_ERR_CAPACITY;

    hipStream_t st = (hipStream_t)stream;
#define NA_TRY(e)                                  \
    do {                                           \
        if ((e) != hipSuccess) {                   \
            (void)hipGetLastError();               \
            return MTS_ERR_HIP;                    \
        }                                          \
    } while (0)
    // state a previous call may have left: everything that must start at zero or at a
    // fixed value, by fill kernels (capturable)
    k_put_desc<<<1, 1, 0, st>>>(sd, d);
    NA_TRY(hipGetLastError());
    NA_TRY(fill_int(st, flags, 1, 0));
    NA_TRY(fill_int(st, tile_obs, 1, 0));
    NA_TRY(fill_int(st, red_done, 2, 0));
    NA_TRY(fill_int(st, count, ncell, 0));
    NA_TRY(fill_int(st, tile_sum, 2 * (int64_t)ntile + 1, 0));
    NA_TRY(fill_int(st, sys_of_cell, ncell, 0));
    NA_TRY(fill_int(st, sys_of, n, 0));

    BinArgs b{};
    b.n = n;
    b.x = x;
    b.sys_of = sys_of;
    b.flags = flags;
    b.ng = 1;
    BinGrid &g = b.g[0];
    g.sd = sd;
    g.ncell = (int)ncell;
    g.cell_of = cell_of;
    g.rank = rank;
    g.count = count;
    g.start = start;
    g.start_loc = start_loc;
    g.tile_sum = tile_sum;
    g.tmp = tmp;
    g.perm = perm;
    g.inv_perm = inv_perm;
    g.xs = xs;
    g.x_ref = nullptr;
    NA_TRY(launch_bin(st, b));

    TripletArgs a{};
    a.ncell = (int)ncell;
    a.cell_map = nullptr;
    a.xs = xs;
    a.start = start;
    a.sd = sd;
    a.sys_of_cell = sys_of_cell;
    a.perm = perm;
    a.pf = pf;
    a.ce = ew ? ce : nullptr;
    a.cc = nullptr;
    a.n = n;
    a.nu = params->nu;
    a.rc2 = rc3 * rc3;
    a.stage_cap = stage_cap;
    a.list_cap = list_cap;
    a.flags = flags;
    a.tile_obs = tile_obs;
    a.any_whole = d.whole;
    NA_TRY(launch_triplet(st, a, fp32, false));
    NA_TRY(launch_triplet_gather(st, n, pf, perm, f3, flags));
    if (ew) {
        ReduceArgs ra{};
        ra.nsys = 1;
        ra.sd = sd;
        ra.ce = ce;
        ra.out = ew;
        ra.stride = 2;
        ra.flags = flags;
        ra.part = part;
        ra.done = red_done;
        ra.chunks = red_chunks(n);
        NA_TRY(launch_reduce(st, ra));
    }
    int hflags = 0;
    NA_TRY(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    NA_TRY(hipStreamSynchronize(st));
#undef NA_TRY
    if (hflags & (kFlagStageOverflow | kFlagListOverflow)) return MTS_ERR_CAPACITY;
    if (hflags & kFlagNonFinite) return MTS_ERR_NONFINITE;
    return MTS_OK;
}
