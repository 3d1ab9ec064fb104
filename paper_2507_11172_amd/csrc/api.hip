// C ABI of the library (declared in include/mts.h): handle life cycle, validation,
// buffer ownership and the host-side sequencing of the r-RESPA loop of Sec. 4.1,
// Algorithm 2.  All device work is enqueued on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mts.h"
#include "common.h"

using namespace mts;


struct mts_system {
    mts_params p{};
    int nsys = 0;
    int64_t n = 0;
    int ncell = 0;
    std::vector<SysDesc> hsd;
    hipStream_t st = nullptr;
    bool fp32 = false;
    int stage_cap = 0, list_cap = 0, pair_cap = 0;
    size_t max_lds = 64 * 1024;  // per-workgroup LDS limit of the device
    double ushift = 0.0;
    std::string err;

    // device buffers (library-owned)
    SysDesc *sd = nullptr;
    int *sys_of = nullptr;       // [n]
    int *sys_of_cell = nullptr;  // [ncell]
    int *cell_of = nullptr, *rank = nullptr, *count = nullptr, *start = nullptr, *perm = nullptr;
    int *perm_tmp = nullptr;     // [n] unordered scatter before ranking
    double *red_part = nullptr;  // [nsys][kRedChunks][6] reduction partials
    double *xs = nullptr;        // [3][n]
    double *f2a = nullptr, *f2b = nullptr, *f3 = nullptr;  // [n][3] force caches
    double *pf = nullptr;        // [14][3][n]
    double *pe = nullptr;        // [n][2]
    double *ce = nullptr;        // [ncell][2]
    long long *cc = nullptr;     // [ncell]
    long long *cnt_sys = nullptr;  // [nsys]
    int *flags = nullptr;
    int *row = nullptr;
    double *e_buf = nullptr;     // [e_rows][nsys][5] energy records of one respa_step
    int64_t e_rows = 0;
    unsigned long long *list_n = nullptr;

    // r-RESPA cycles run on an internal stream, optionally replayed from captured graphs
    hipStream_t ist = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    bool use_graph = true;
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [energies][F2 parity]
    double *xi = nullptr, *vi = nullptr;  // internal copies of x and v, [n][3]

    // optional per-launch HIP-event timing of the two force kernels (0: triplet, 1: pair)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool[2];
    size_t ev_used[2] = {0, 0};
};

namespace {

mts_status fail(mts_system *s, mts_status code, const std::string &msg) {
    if (s) s->err = msg;
    return code;
}

mts_status hip_fail(mts_system *s, hipError_t e, const char *what) {
    return fail(s, MTS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(sys, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(sys, _e, #expr); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

mts_status validate_params(const mts_params *p, std::string &msg) {
    if (!p) { msg = "params is NULL"; return MTS_ERR_INVALID_ARG; }
    if (!std::isfinite(p->epsilon) || p->epsilon < 0.0) { msg = "epsilon must be finite and >= 0"; return MTS_ERR_INVALID_ARG; }
    if (!finite_pos(p->sigma)) { msg = "sigma must be > 0"; return MTS_ERR_INVALID_ARG; }
    if (!finite_pos(p->rc_pair) || !finite_pos(p->rc_triplet)) { msg = "cutoffs must be > 0"; return MTS_ERR_INVALID_ARG; }
    if (!std::isfinite(p->nu)) { msg = "nu must be finite"; return MTS_ERR_INVALID_ARG; }
    if (!finite_pos(p->mass)) { msg = "mass must be > 0"; return MTS_ERR_INVALID_ARG; }
    if (!finite_pos(p->dt)) { msg = "dt must be > 0"; return MTS_ERR_INVALID_ARG; }
    if (p->k < 1) { msg = "k (step-size factor) must be >= 1"; return MTS_ERR_INVALID_ARG; }
    if (p->precision != MTS_FP64 && p->precision != MTS_FP32) { msg = "unknown precision"; return MTS_ERR_INVALID_ARG; }
    if (p->reserved != 0) { msg = "reserved must be 0"; return MTS_ERR_INVALID_ARG; }
    return MTS_OK;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Tile capacities.  A cell of volume h^3 holds about rho h^3 particles; sizing assumes a
// local density of max(0.9, 1.2 x the system's mean), which covers LJ liquids and
// crystals near the densities of the paper's scenarios, including a liquid slab inside
// a dilute box.  The triplet tile holds the 14 cells of the forward half stencil, the
// pair tile all 27 cells, and a forward-neighbour list about half a cutoff sphere.
// Overflow is detected on the device, reported by mts_sync, and doubles the capacity
// for the next call.
void size_tiles(mts_system *s) {
    double need = 0.0, nl = 0.0;
    const double rc3 = s->p.rc_triplet;
    for (const SysDesc &d : s->hsd) {
        const double vol = d.L[0] * d.L[1] * d.L[2];
        const double rho = std::max(0.9, 1.2 * (double)d.n / vol);
        const double cellv = (d.L[0] / d.nc[0]) * (d.L[1] / d.nc[1]) * (d.L[2] / d.nc[2]);
        need = std::max(need, rho * cellv);
        nl = std::max(nl, rho * (2.0 / 3.0) * M_PI * rc3 * rc3 * rc3);
    }
    s->stage_cap = std::min(2048, round_up((int)std::ceil(kNumHalf * need * 1.1) + 16, 32));
    s->pair_cap = std::min(2048, round_up((int)std::ceil(kNumFull * need * 1.1) + 16, 32));
    s->list_cap = std::min(1024, round_up((int)std::ceil(1.6 * nl) + 16, 32));
}

mts_status alloc_all(mts_system *s) {
    const int64_t n = s->n;
    HIP_TRY(s, dalloc(&s->sd, s->nsys));
    HIP_TRY(s, dalloc(&s->sys_of, n));
    HIP_TRY(s, dalloc(&s->sys_of_cell, s->ncell));
    HIP_TRY(s, dalloc(&s->cell_of, n));
    HIP_TRY(s, dalloc(&s->rank, n));
    HIP_TRY(s, dalloc(&s->count, s->ncell));
    HIP_TRY(s, dalloc(&s->start, (size_t)s->ncell + 1));
    HIP_TRY(s, dalloc(&s->perm, n));
    HIP_TRY(s, dalloc(&s->perm_tmp, n));
    HIP_TRY(s, dalloc(&s->red_part, (size_t)s->nsys * kRedChunks * 6));
    HIP_TRY(s, dalloc(&s->xs, 3 * n));
    HIP_TRY(s, dalloc(&s->f2a, 3 * n));
    HIP_TRY(s, dalloc(&s->f2b, 3 * n));
    HIP_TRY(s, dalloc(&s->f3, 3 * n));
    HIP_TRY(s, dalloc(&s->pf, (size_t)kNumHalf * 3 * n));
    HIP_TRY(s, dalloc(&s->pe, 2 * n));
    HIP_TRY(s, dalloc(&s->ce, 2 * (size_t)s->ncell));
    HIP_TRY(s, dalloc(&s->cc, s->ncell));
    HIP_TRY(s, dalloc(&s->cnt_sys, s->nsys));
    HIP_TRY(s, dalloc(&s->flags, 1));
    HIP_TRY(s, dalloc(&s->row, 1));
    HIP_TRY(s, dalloc(&s->list_n, 1));
    HIP_TRY(s, dalloc(&s->xi, 3 * n));
    HIP_TRY(s, dalloc(&s->vi, 3 * n));
    HIP_TRY(s, hipStreamCreateWithFlags(&s->ist, hipStreamNonBlocking));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));

    std::vector<int> so(n > 0 ? n : 1), soc(s->ncell);
    for (int q = 0; q < s->nsys; ++q) {
        const SysDesc &d = s->hsd[q];
        for (int64_t i = 0; i < d.n; ++i) so[d.p0 + i] = q;
        for (int c = 0; c < d.ncell; ++c) soc[d.cell0 + c] = q;
    }
    HIP_TRY(s, hipMemcpy(s->sd, s->hsd.data(), sizeof(SysDesc) * s->nsys, hipMemcpyHostToDevice));
    if (n > 0) HIP_TRY(s, hipMemcpy(s->sys_of, so.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(s->sys_of_cell, soc.data(), sizeof(int) * s->ncell, hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemset(s->count, 0, sizeof(int) * s->ncell));
    HIP_TRY(s, hipMemset(s->flags, 0, sizeof(int)));
    HIP_TRY(s, hipMemset(s->pf, 0, sizeof(double) * kNumHalf * 3 * (n > 0 ? n : 1)));
    return MTS_OK;
}

// Records a start event before a timed kernel launch; returns the slot or -1.
long timer_begin(mts_system *s, int cls) {
    if (!s->timing) return -1;
    std::vector<hipEvent_t> &pool = s->ev_pool[cls];
    const size_t slot = s->ev_used[cls];
    if (pool.size() < slot + 2) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
        pool.push_back(a);
        pool.push_back(b);
    }
    if (hipEventRecord(pool[slot], s->st) != hipSuccess) return -1;
    s->ev_used[cls] = slot + 2;
    return (long)slot;
}

void timer_end(mts_system *s, int cls, long slot) {
    if (slot >= 0) (void)hipEventRecord(s->ev_pool[cls][slot + 1], s->st);
}

void drop_graphs(mts_system *s) {
    for (auto &g : s->gexec)
        for (hipGraphExec_t &e : g)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
}

void free_all(mts_system *s) {
    drop_graphs(s);
    if (s->ev_in) (void)hipEventDestroy(s->ev_in);
    if (s->ev_out) (void)hipEventDestroy(s->ev_out);
    if (s->ist) (void)hipStreamDestroy(s->ist);
    for (int c = 0; c < 2; ++c)
        for (hipEvent_t e : s->ev_pool[c]) (void)hipEventDestroy(e);
    void *ptrs[] = {s->sd, s->sys_of, s->sys_of_cell, s->cell_of, s->rank, s->count, s->start,
                    s->perm, s->xs, s->f2a, s->f2b, s->f3, s->pf, s->pe, s->ce, s->cc,
                    s->cnt_sys, s->flags, s->row, s->e_buf, s->list_n, s->perm_tmp,
                    s->red_part, s->xi, s->vi};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

// ---- enqueue helpers
mts_status enqueue_bin(mts_system *s, const double *x) {
    HIP_TRY(s, launch_bin_count(s->st, s->n, x, s->sd, s->sys_of, s->cell_of, s->rank, s->count,
                                s->flags));
    HIP_TRY(s, launch_scan(s->st, s->ncell, s->count, s->start, s->n));
    HIP_TRY(s, launch_bin_scatter(s->st, s->n, s->cell_of, s->rank, s->start, s->perm_tmp));
    HIP_TRY(s, launch_rank_gather(s->st, s->n, s->perm_tmp, s->cell_of, s->start, x, s->sd,
                                  s->sys_of, s->perm, s->xs));
    return MTS_OK;
}

mts_status enqueue_pair(mts_system *s, double *f2) {
    PairArgs a{};
    a.ncell = s->ncell;
    a.sys_of_cell = s->sys_of_cell;
    a.stage_cap = s->pair_cap;
    a.n = s->n;
    a.xs = s->xs;
    a.perm = s->perm;
    a.start = s->start;
    a.sd = s->sd;
    a.sys_of = s->sys_of;
    a.f = f2;
    a.pe = s->pe;
    a.eps = s->p.epsilon;
    a.sigma2 = s->p.sigma * s->p.sigma;
    a.rc2 = s->p.rc_pair * s->p.rc_pair;
    a.ushift = s->ushift;
    a.flags = s->flags;
    const long ts = timer_begin(s, 1);
    HIP_TRY(s, launch_pair(s->st, a, s->fp32));
    timer_end(s, 1, ts);
    return MTS_OK;
}

mts_status enqueue_triplet(mts_system *s, double *f3, int *list_ijk, long long list_rows) {
    TripletArgs a{};
    a.ncell = s->ncell;
    a.xs = s->xs;
    a.start = s->start;
    a.sd = s->sd;
    a.sys_of_cell = s->sys_of_cell;
    a.perm = s->perm;
    a.pf = s->pf;
    a.ce = s->ce;
    a.cc = s->cc;
    a.n = s->n;
    a.nu = s->p.nu;
    a.rc2 = s->p.rc_triplet * s->p.rc_triplet;
    a.stage_cap = s->stage_cap;
    a.list_cap = s->list_cap;
    a.flags = s->flags;
    a.list_ijk = list_ijk;
    a.list_n = s->list_n;
    a.list_rows = list_rows;
    const long ts = timer_begin(s, 0);
    HIP_TRY(s, launch_triplet(s->st, a, s->fp32, list_ijk != nullptr));
    timer_end(s, 0, ts);
    if (f3) HIP_TRY(s, launch_triplet_gather(s->st, s->n, s->pf, s->perm, f3, s->flags));
    return MTS_OK;
}

mts_status enqueue_reduce(mts_system *s, const double *v, bool pair, bool trip, double *out,
                          int stride, const int *row, long long *count_out) {
    ReduceArgs a{};
    a.nsys = s->nsys;
    a.sd = s->sd;
    a.v = v;
    a.half_mass = 0.5 * s->p.mass;
    a.pe = pair ? s->pe : nullptr;
    a.ce = trip ? s->ce : nullptr;
    a.cc = trip ? s->cc : nullptr;
    a.out = out;
    a.stride = stride;
    a.count_out = count_out;
    a.flags = s->flags;
    a.row = row;
    a.part = s->red_part;
    HIP_TRY(s, launch_reduce(s->st, a));
    return MTS_OK;
}

#define MTS_TRY(expr)                 \
    do {                              \
        mts_status _r = (expr);       \
        if (_r != MTS_OK) return _r;  \
    } while (0)

double lj_energy(double r2, double eps, double sigma) {
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

}  // namespace

extern "C" {

const char *mts_status_string(int32_t status) {
    switch (status) {
        case MTS_OK: return "MTS_OK";
        case MTS_ERR_INVALID_ARG: return "MTS_ERR_INVALID_ARG";
        case MTS_ERR_BOX_TOO_SMALL: return "MTS_ERR_BOX_TOO_SMALL";
        case MTS_ERR_NOT_MULTIPLE_OF_K: return "MTS_ERR_NOT_MULTIPLE_OF_K";
        case MTS_ERR_CAPACITY: return "MTS_ERR_CAPACITY";
        case MTS_ERR_NONFINITE: return "MTS_ERR_NONFINITE";
        case MTS_ERR_HIP: return "MTS_ERR_HIP";
        case MTS_ERR_OOM: return "MTS_ERR_OOM";
        case MTS_ERR_UNSUPPORTED: return "MTS_ERR_UNSUPPORTED";
        default: return "unknown status";
    }
}

mts_status mts_init_system(const mts_params *params, int32_t n_systems, const int64_t *n_particles,
                           const double *box, void *stream, mts_system **out) {
    if (!out) return MTS_ERR_INVALID_ARG;
    *out = nullptr;
    std::string msg;
    mts_status v = validate_params(params, msg);
    if (v != MTS_OK) return v;
    if (n_systems < 1 || !n_particles || !box) return MTS_ERR_INVALID_ARG;
    mts_system *s = new mts_system();
    s->p = *params;
    s->nsys = n_systems;
    s->st = (hipStream_t)stream;
    s->fp32 = params->precision == MTS_FP32;
    const double rc_max = std::max(params->rc_pair, params->rc_triplet);
    // cells strictly wider than the largest cutoff, with margin for rounding, so that any
    // interacting pair lies in adjacent cells
    const double hmin = rc_max * (1.0 + 1e-9);
    int64_t p0 = 0;
    int64_t cell0 = 0;
    for (int q = 0; q < n_systems; ++q) {
        SysDesc d{};
        if (n_particles[q] < 0) { delete s; return MTS_ERR_INVALID_ARG; }
        for (int k = 0; k < 3; ++k) {
            const double L = box[3 * q + k];
            if (!finite_pos(L)) { delete s; return MTS_ERR_INVALID_ARG; }
            if (!(L > 2.0 * hmin)) { delete s; return MTS_ERR_BOX_TOO_SMALL; }
            d.L[k] = L;
            d.nc[k] = (int)std::floor(L / hmin);
            if (d.nc[k] < 2) { delete s; return MTS_ERR_BOX_TOO_SMALL; }
            d.q[k] = (double)d.nc[k] / L;
        }
        d.ncell = d.nc[0] * d.nc[1] * d.nc[2];
        d.cell0 = (int)cell0;
        d.p0 = p0;
        d.n = n_particles[q];
        p0 += d.n;
        cell0 += d.ncell;
        s->hsd.push_back(d);
    }
    if (p0 >= (int64_t)1 << 30 || cell0 >= (int64_t)1 << 30) { delete s; return MTS_ERR_UNSUPPORTED; }
    s->n = p0;
    s->ncell = (int)cell0;
    s->ushift = params->lj_energy_shift
                    ? lj_energy(params->rc_pair * params->rc_pair, params->epsilon, params->sigma)
                    : 0.0;
    size_tiles(s);
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            s->max_lds = (size_t)lds;
        // keep room for the kernels' static LDS
        s->max_lds = s->max_lds > 1024 ? s->max_lds - 1024 : s->max_lds;
        if (configure_kernel_lds(s->max_lds) != hipSuccess) s->max_lds = 64 * 1024 - 1024;
        (void)hipGetLastError();  // do not leave a failed attribute call as a sticky error
    }
    if (triplet_lds_bytes(s->stage_cap, s->list_cap) > s->max_lds ||
        pair_lds_bytes(s->pair_cap) > s->max_lds) {
        free_all(s);
        delete s;
        return MTS_ERR_UNSUPPORTED;
    }
    mts_status a = alloc_all(s);
    if (a != MTS_OK) {
        free_all(s);
        delete s;
        return a == MTS_ERR_HIP ? MTS_ERR_OOM : a;
    }
    *out = s;
    return MTS_OK;
}

void mts_destroy_system(mts_system *sys) {
    if (!sys) return;
    if (sys->ist) (void)hipStreamSynchronize(sys->ist);
    (void)hipStreamSynchronize(sys->st);
    free_all(sys);
    delete sys;
}

mts_status mts_build_cells(mts_system *sys, const double *x) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if (!x && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x is NULL");
    return enqueue_bin(sys, x);
}

mts_status mts_compute_pair_forces(mts_system *sys, const double *x, double *f2, double *ew) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !f2) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or f2 is NULL");
    MTS_TRY(enqueue_bin(sys, x));
    MTS_TRY(enqueue_pair(sys, f2));
    if (ew) MTS_TRY(enqueue_reduce(sys, nullptr, true, false, ew, 2, nullptr, nullptr));
    return MTS_OK;
}

mts_status mts_compute_triplet_forces(mts_system *sys, const double *x, double *f3, double *ew) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !f3) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or f3 is NULL");
    MTS_TRY(enqueue_bin(sys, x));
    MTS_TRY(enqueue_triplet(sys, f3, nullptr, 0));
    if (ew) MTS_TRY(enqueue_reduce(sys, nullptr, false, true, ew, 2, nullptr, nullptr));
    return MTS_OK;
}

// One outer cycle of Algorithm 2 on the internal copies xi, vi: k inner steps (F3 half
// kick at the first, drift + wrap, binning, F2, F2 kick), then F3 at the full step, its
// half kick and, if requested, the energy record.  f2a holds F2 of the cycle's first
// position; after the cycle F2 of the last position is in f2a when k is even, f2b when odd.
mts_status enqueue_cycle(mts_system *s, double *f2a, double *f2b, bool energies) {
    const int k = s->p.k;
    const int64_t n3 = 3 * s->n;
    const double dt = s->p.dt, m = s->p.mass;
    const double c3 = (dt * (double)k) / (2.0 * m);
    const double cx = (dt * dt) / (2.0 * m);
    const double c2 = dt / (2.0 * m);
    double *f2cur = f2a, *f2nxt = f2b;
    for (int i = 0; i < k; ++i) {
        if (i == 0) HIP_TRY(s, launch_kick(s->st, n3, s->vi, s->f3, c3));
        HIP_TRY(s, launch_drift(s->st, s->n, s->xi, s->vi, f2cur, dt, cx, s->sd, s->sys_of));
        MTS_TRY(enqueue_bin(s, s->xi));
        MTS_TRY(enqueue_pair(s, f2nxt));
        HIP_TRY(s, launch_kick2(s->st, n3, s->vi, f2cur, f2nxt, c2));
        std::swap(f2cur, f2nxt);
    }
    MTS_TRY(enqueue_triplet(s, s->f3, nullptr, 0));
    HIP_TRY(s, launch_kick(s->st, n3, s->vi, s->f3, c3));
    if (energies) {
        MTS_TRY(enqueue_reduce(s, s->vi, true, true, s->e_buf, kNE, s->row, nullptr));
        HIP_TRY(s, launch_bump_row(s->st, s->row));
    }
    return MTS_OK;
}

// Captures one cycle into an executable graph (kernels only: no memset or copy nodes).
mts_status capture_cycle(mts_system *s, bool energies, int parity) {
    double *fa = parity ? s->f2b : s->f2a, *fb = parity ? s->f2a : s->f2b;
    HIP_TRY(s, hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    mts_status r = enqueue_cycle(s, fa, fb, energies);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->st, &g);
    if (r != MTS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(s, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->gexec[energies][parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
    return MTS_OK;
}

mts_status respa_internal(mts_system *s, double *x, double *v, int64_t n_iter, double *e_full) {
    const int k = s->p.k;
    const int64_t cycles = n_iter / k;
    const bool energies = e_full != nullptr;
    const int64_t bytes = 3 * s->n * (int64_t)sizeof(double);
    if (energies && s->e_rows < cycles + 1) {
        // grow the energy record buffer; graphs holding the old pointer are dropped
        drop_graphs(s);
        if (s->e_buf) HIP_TRY(s, hipFree(s->e_buf));
        s->e_buf = nullptr;
        s->e_rows = 0;
        HIP_TRY(s, dalloc(&s->e_buf, (size_t)(cycles + 1) * s->nsys * kNE));
        s->e_rows = cycles + 1;
    }
    if (bytes > 0) {
        HIP_TRY(s, hipMemcpyAsync(s->xi, x, bytes, hipMemcpyDeviceToDevice, s->st));
        HIP_TRY(s, hipMemcpyAsync(s->vi, v, bytes, hipMemcpyDeviceToDevice, s->st));
    }
    // Algorithm 2, lines 1-2: F2(x^0), F3(x^0); energies of x^0 in row 0
    MTS_TRY(enqueue_bin(s, s->xi));
    MTS_TRY(enqueue_pair(s, s->f2a));
    MTS_TRY(enqueue_triplet(s, s->f3, nullptr, 0));
    if (energies) {
        HIP_TRY(s, launch_set_int(s->st, s->row, 0));
        MTS_TRY(enqueue_reduce(s, s->vi, true, true, s->e_buf, kNE, s->row, nullptr));
        HIP_TRY(s, launch_bump_row(s->st, s->row));
    }
    const bool graph = s->use_graph && !s->timing;
    for (int64_t c = 0; c < cycles; ++c) {
        const int parity = (k & 1) ? (int)(c & 1) : 0;
        if (graph) {
            if (!s->gexec[energies][parity]) MTS_TRY(capture_cycle(s, energies, parity));
            HIP_TRY(s, hipGraphLaunch(s->gexec[energies][parity], s->st));
        } else {
            MTS_TRY(enqueue_cycle(s, parity ? s->f2b : s->f2a, parity ? s->f2a : s->f2b, energies));
        }
    }
    if (bytes > 0) {
        HIP_TRY(s, hipMemcpyAsync(x, s->xi, bytes, hipMemcpyDeviceToDevice, s->st));
        HIP_TRY(s, hipMemcpyAsync(v, s->vi, bytes, hipMemcpyDeviceToDevice, s->st));
    }
    if (energies)
        HIP_TRY(s, hipMemcpyAsync(e_full, s->e_buf, sizeof(double) * (size_t)(cycles + 1) * s->nsys * kNE,
                                  hipMemcpyDeviceToDevice, s->st));
    return MTS_OK;
}

mts_status mts_respa_step(mts_system *sys, double *x, double *v, int64_t n_iter, double *e_full) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !v) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or v is NULL");
    if (n_iter < 0) return fail(sys, MTS_ERR_INVALID_ARG, "n_iter < 0");
    if (n_iter % sys->p.k != 0)
        return fail(sys, MTS_ERR_NOT_MULTIPLE_OF_K, "n_iter must be a multiple of k (Sec. 4.1)");
    // run on the internal stream, ordered after and before the caller's stream
    hipStream_t user = sys->st;
    HIP_TRY(sys, hipEventRecord(sys->ev_in, user));
    HIP_TRY(sys, hipStreamWaitEvent(sys->ist, sys->ev_in, 0));
    sys->st = sys->ist;
    mts_status r = respa_internal(sys, x, v, n_iter, e_full);
    sys->st = user;
    HIP_TRY(sys, hipEventRecord(sys->ev_out, sys->ist));
    HIP_TRY(sys, hipStreamWaitEvent(user, sys->ev_out, 0));
    return r;
}

mts_status mts_set_option(mts_system *sys, int32_t option, int64_t value) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    switch (option) {
        case MTS_OPT_CYCLE_GRAPH:
            sys->use_graph = value != 0;
            return MTS_OK;
        default:
            return fail(sys, MTS_ERR_INVALID_ARG, "unknown option");
    }
}

mts_status mts_sync(mts_system *sys) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    HIP_TRY(sys, hipStreamSynchronize(sys->ist));
    HIP_TRY(sys, hipStreamSynchronize(sys->st));
    int flags = 0;
    HIP_TRY(sys, hipMemcpy(&flags, sys->flags, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(sys, hipMemset(sys->flags, 0, sizeof(int)));
    if (flags & (kFlagStageOverflow | kFlagListOverflow)) {
        const int old_s = sys->stage_cap, old_l = sys->list_cap, old_p = sys->pair_cap;
        if (flags & kFlagStageOverflow) {
            sys->stage_cap = std::min(4096, 2 * sys->stage_cap);
            sys->pair_cap = std::min(4096, 2 * sys->pair_cap);
        }
        if (flags & kFlagListOverflow) sys->list_cap = std::min(2048, 2 * sys->list_cap);
        if (triplet_lds_bytes(sys->stage_cap, sys->list_cap) > sys->max_lds) {
            sys->stage_cap = old_s;
            sys->list_cap = old_l;
        }
        if (pair_lds_bytes(sys->pair_cap) > sys->max_lds) sys->pair_cap = old_p;
        drop_graphs(sys);  // captured launches carry the old tile sizes
        char buf[200];
        snprintf(buf, sizeof buf,
                 "capacity overflow (flags %d): triplet tile %d -> %d, pair tile %d -> %d, "
                 "neighbour list %d -> %d; results since the last sync are invalid",
                 flags, old_s, sys->stage_cap, old_p, sys->pair_cap, old_l, sys->list_cap);
        return fail(sys, MTS_ERR_CAPACITY, buf);
    }
    if (flags & kFlagNonFinite) return fail(sys, MTS_ERR_NONFINITE, "non-finite force or energy");
    return MTS_OK;
}

const char *mts_last_error(const mts_system *sys) { return sys ? sys->err.c_str() : ""; }

mts_status mts_get_grid(const mts_system *sys, int32_t system, int32_t n_cells[3]) {
    if (!sys || !n_cells || system < 0 || system >= sys->nsys) return MTS_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) n_cells[k] = sys->hsd[system].nc[k];
    return MTS_OK;
}

mts_status mts_get_cell_index(mts_system *sys, int32_t *cell) {
    if (!sys || (!cell && sys->n > 0)) return MTS_ERR_INVALID_ARG;
    HIP_TRY(sys, launch_local_cell_index(sys->st, sys->n, sys->cell_of, sys->sd, sys->sys_of, cell));
    return MTS_OK;
}

mts_status mts_count_triplets(mts_system *sys, const double *x, int64_t *count) {
    if (!sys || !count || (!x && sys->n > 0)) return MTS_ERR_INVALID_ARG;
    MTS_TRY(enqueue_bin(sys, x));
    MTS_TRY(enqueue_triplet(sys, nullptr, nullptr, 0));
    MTS_TRY(enqueue_reduce(sys, nullptr, false, true, nullptr, 2, nullptr, sys->cnt_sys));
    std::vector<long long> c(sys->nsys);
    HIP_TRY(sys, hipMemcpyAsync(c.data(), sys->cnt_sys, sizeof(long long) * sys->nsys,
                                hipMemcpyDeviceToHost, sys->st));
    MTS_TRY(mts_sync(sys));
    int64_t t = 0;
    for (long long v : c) t += v;
    *count = t;
    return MTS_OK;
}

mts_status mts_list_triplets(mts_system *sys, const double *x, int32_t *ijk, int64_t cap,
                             int64_t *n) {
    if (!sys || !n || cap < 0 || (!x && sys->n > 0)) return MTS_ERR_INVALID_ARG;
    if (!ijk || cap == 0) return mts_count_triplets(sys, x, n);
    HIP_TRY(sys, hipMemsetAsync(sys->list_n, 0, sizeof(unsigned long long), sys->st));
    MTS_TRY(enqueue_bin(sys, x));
    MTS_TRY(enqueue_triplet(sys, nullptr, ijk, cap));
    unsigned long long total = 0;
    HIP_TRY(sys, hipMemcpyAsync(&total, sys->list_n, sizeof(unsigned long long), hipMemcpyDeviceToHost, sys->st));
    MTS_TRY(mts_sync(sys));
    *n = (int64_t)total;
    return MTS_OK;
}

mts_status mts_enable_kernel_timing(mts_system *sys, int32_t enable) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    HIP_TRY(sys, hipStreamSynchronize(sys->ist));
    HIP_TRY(sys, hipStreamSynchronize(sys->st));
    sys->timing = enable != 0;
    sys->ev_used[0] = sys->ev_used[1] = 0;
    return MTS_OK;
}

mts_status mts_kernel_times(mts_system *sys, int64_t launches[2], double ms[2]) {
    if (!sys || !launches || !ms) return MTS_ERR_INVALID_ARG;
    HIP_TRY(sys, hipStreamSynchronize(sys->ist));
    HIP_TRY(sys, hipStreamSynchronize(sys->st));
    for (int c = 0; c < 2; ++c) {
        double tot = 0.0;
        for (size_t q = 0; q + 1 < sys->ev_used[c]; q += 2) {
            float t = 0.0f;
            HIP_TRY(sys, hipEventElapsedTime(&t, sys->ev_pool[c][q], sys->ev_pool[c][q + 1]));
            tot += t;
        }
        launches[c] = (int64_t)(sys->ev_used[c] / 2);
        ms[c] = tot;
        sys->ev_used[c] = 0;
    }
    return MTS_OK;
}

}  // extern "C"
