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
    int pair_lanes = 8;
    int stage_cap = 0, list_cap = 0;
    double ushift = 0.0;
    std::string err;

    // device buffers (library-owned)
    SysDesc *sd = nullptr;
    int *sys_of = nullptr;       // [n]
    int *sys_of_cell = nullptr;  // [ncell]
    int *cell_of = nullptr, *rank = nullptr, *count = nullptr, *start = nullptr, *perm = nullptr;
    double *xs = nullptr;        // [3][n]
    double *f2a = nullptr, *f2b = nullptr, *f3 = nullptr;  // [n][3] force caches
    double *pf = nullptr;        // [14][3][n]
    double *pe = nullptr;        // [n][2]
    double *ce = nullptr;        // [ncell][2]
    long long *cc = nullptr;     // [ncell]
    long long *cnt_sys = nullptr;  // [nsys]
    int *flags = nullptr;
    int *row = nullptr;
    double *e_buf = nullptr;     // [rows][nsys][5]
    int64_t e_rows = 0;
    unsigned long long *list_n = nullptr;

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

// Tile capacities.  The staged half stencil holds 14 cells; a cell of volume h^3 holds
// about rho h^3 particles.  Sizing assumes a local density of at least 1.25 (above any
// LJ liquid or solid at these temperatures) so that slabs and crystals fit; overflow is
// detected on the device and doubles the capacity for the next call.
void size_tiles(mts_system *s) {
    double need = 0.0, nl = 0.0;
    const double rc3 = s->p.rc_triplet;
    for (const SysDesc &d : s->hsd) {
        const double vol = d.L[0] * d.L[1] * d.L[2];
        const double rho = std::max(1.25, 1.5 * (double)d.n / vol);
        const double cellv = (d.L[0] / d.nc[0]) * (d.L[1] / d.nc[1]) * (d.L[2] / d.nc[2]);
        need = std::max(need, kNumHalf * rho * cellv);
        nl = std::max(nl, rho * (4.0 / 3.0) * M_PI * rc3 * rc3 * rc3);  // full sphere: 2x the forward half
    }
    s->stage_cap = std::min(2048, round_up((int)std::ceil(need * 1.15) + 32, 64));
    s->list_cap = std::min(1024, round_up((int)std::ceil(nl) + 16, 32));
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

void free_all(mts_system *s) {
    for (int c = 0; c < 2; ++c)
        for (hipEvent_t e : s->ev_pool[c]) (void)hipEventDestroy(e);
    void *ptrs[] = {s->sd, s->sys_of, s->sys_of_cell, s->cell_of, s->rank, s->count, s->start,
                    s->perm, s->xs, s->f2a, s->f2b, s->f3, s->pf, s->pe, s->ce, s->cc,
                    s->cnt_sys, s->flags, s->row, s->e_buf, s->list_n};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

// ---- enqueue helpers
mts_status enqueue_bin(mts_system *s, const double *x) {
    HIP_TRY(s, launch_bin_count(s->st, s->n, x, s->sd, s->sys_of, s->cell_of, s->rank, s->count,
                                s->flags));
    HIP_TRY(s, launch_scan(s->st, s->ncell, s->count, s->start, s->n));
    HIP_TRY(s, launch_bin_scatter(s->st, s->n, s->cell_of, s->rank, s->start, s->perm));
    HIP_TRY(s, launch_cell_sort(s->st, s->ncell, s->start, s->perm, s->count));
    HIP_TRY(s, launch_gather_sorted(s->st, s->n, x, s->perm, s->sd, s->sys_of, s->xs));
    return MTS_OK;
}

mts_status enqueue_pair(mts_system *s, double *f2) {
    PairArgs a{};
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
    HIP_TRY(s, launch_pair(s->st, a, s->fp32, s->pair_lanes));
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
    if (triplet_lds_bytes(s->stage_cap, s->list_cap) > 64 * 1024) {
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

mts_status mts_respa_step(mts_system *sys, double *x, double *v, int64_t n_iter, double *e_full) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !v) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or v is NULL");
    if (n_iter < 0) return fail(sys, MTS_ERR_INVALID_ARG, "n_iter < 0");
    const int k = sys->p.k;
    if (n_iter % k != 0)
        return fail(sys, MTS_ERR_NOT_MULTIPLE_OF_K, "n_iter must be a multiple of k (Sec. 4.1)");
    const int64_t n3 = 3 * sys->n;
    const double dt = sys->p.dt, m = sys->p.mass;
    const double c3 = (dt * (double)k) / (2.0 * m);
    const double cx = (dt * dt) / (2.0 * m);
    const double c2 = dt / (2.0 * m);
    int *row = nullptr;
    double *eout = nullptr;
    if (e_full) {
        HIP_TRY(sys, hipMemsetAsync(sys->row, 0, sizeof(int), sys->st));
        row = sys->row;
        eout = e_full;
    }
    // Algorithm 2, lines 1-2: F2(x^0), F3(x^0)
    double *f2cur = sys->f2a, *f2nxt = sys->f2b;
    MTS_TRY(enqueue_bin(sys, x));
    MTS_TRY(enqueue_pair(sys, f2cur));
    MTS_TRY(enqueue_triplet(sys, sys->f3, nullptr, 0));
    if (eout) {
        MTS_TRY(enqueue_reduce(sys, v, true, true, eout, kNE, row, nullptr));
        HIP_TRY(sys, launch_bump_row(sys->st, sys->row));
    }
    for (int64_t i = 0; i < n_iter; ++i) {
        if (i % k == 0) HIP_TRY(sys, launch_kick(sys->st, n3, v, sys->f3, c3));
        HIP_TRY(sys, launch_drift(sys->st, sys->n, x, v, f2cur, dt, cx, sys->sd, sys->sys_of));
        MTS_TRY(enqueue_bin(sys, x));
        MTS_TRY(enqueue_pair(sys, f2nxt));
        HIP_TRY(sys, launch_kick2(sys->st, n3, v, f2cur, f2nxt, c2));
        std::swap(f2cur, f2nxt);
        if ((i + 1) % k == 0) {
            MTS_TRY(enqueue_triplet(sys, sys->f3, nullptr, 0));
            HIP_TRY(sys, launch_kick(sys->st, n3, v, sys->f3, c3));
            if (eout) {
                MTS_TRY(enqueue_reduce(sys, v, true, true, eout, kNE, row, nullptr));
                HIP_TRY(sys, launch_bump_row(sys->st, sys->row));
            }
        }
    }
    // keep the F2 cache that belongs to the final x in f2a for the next call's reuse
    if (f2cur != sys->f2a) std::swap(sys->f2a, sys->f2b);
    return MTS_OK;
}

mts_status mts_sync(mts_system *sys) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    HIP_TRY(sys, hipStreamSynchronize(sys->st));
    int flags = 0;
    HIP_TRY(sys, hipMemcpy(&flags, sys->flags, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(sys, hipMemset(sys->flags, 0, sizeof(int)));
    if (flags & (kFlagStageOverflow | kFlagListOverflow)) {
        const int old_s = sys->stage_cap, old_l = sys->list_cap;
        if (flags & kFlagStageOverflow) sys->stage_cap = std::min(4096, 2 * sys->stage_cap);
        if (flags & kFlagListOverflow) sys->list_cap = std::min(2048, 2 * sys->list_cap);
        if (triplet_lds_bytes(sys->stage_cap, sys->list_cap) > 64 * 1024) {
            sys->stage_cap = old_s;
            sys->list_cap = old_l;
        }
        char buf[160];
        snprintf(buf, sizeof buf,
                 "capacity overflow (flags %d): tile %d -> %d, neighbour list %d -> %d; "
                 "results since the last sync are invalid",
                 flags, old_s, sys->stage_cap, old_l, sys->list_cap);
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
    HIP_TRY(sys, hipStreamSynchronize(sys->st));
    sys->timing = enable != 0;
    sys->ev_used[0] = sys->ev_used[1] = 0;
    return MTS_OK;
}

mts_status mts_kernel_times(mts_system *sys, int64_t launches[2], double ms[2]) {
    if (!sys || !launches || !ms) return MTS_ERR_INVALID_ARG;
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
