// C ABI of the library (declared in include/mts.h): handle life cycle, validation,
// buffer ownership and the host-side sequencing of the r-RESPA loop of Sec. 4.1,
// Algorithm 2.
//
// Two linked-cell grids are kept per system:
//   * the triplet grid, cell edge >= rc_triplet, used by the triplet kernel;
//   * the pair grid, cell edge >= rc_pair + skin, used to build a Verlet pair list.
// Between two full steps of r-RESPA the particles move far less than half the skin, so
// the pair list built at a full step holds every pair within rc_pair for the next k
// inner steps; each inner step is then one launch of the list force kernel with the
// update fused behind it, instead of a full rebinning.  A particle that moves more than
// half the skin raises a device flag that mts_sync reports (the list is rebuilt at every
// full step anyway).  Nested r-RESPA (k_outer > 1) runs cycles of k steps the same way; at
// the end of a cycle the inner triplet class is evaluated, at the end of every k_outer-th
// cycle instead the whole cutoff set with per-class weights (see F3Mode).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mts.h"
#include "common.h"

using namespace mts;

namespace {

// One linked-cell binning of all systems.
struct Grid {
    std::vector<SysDesc> hsd;
    SysDesc *sd = nullptr;
    int ncell = 0;
    int *sys_of_cell = nullptr;   // [ncell]
    int *cell_of = nullptr;       // [n] input order
    int *rank = nullptr;          // [n] atomic arrival rank in the cell
    int *count = nullptr;         // [ncell] histogram (kept zero between binnings)
    int *start = nullptr;         // [ncell + 1]
    int *start_loc = nullptr;     // [ncell] tile-local prefix of the scan
    int *tile_sum = nullptr;      // [2 ntile + 1] scan tile totals, offsets and counter
    int *perm_tmp = nullptr;      // [n] unordered scatter
    int *perm = nullptr;          // [n] sorted -> input
    int *inv_perm = nullptr;      // [n] input -> sorted
    Pos4 *xs = nullptr;           // [n] sorted wrapped positions
    Pos4 *xs2 = nullptr;          // [n] second position buffer (pair grid: list steps)
};

// Tunable choices of a handle (see mts_tuning in mts.h).
struct Config {
    double skin = 0.0;            // pair-list skin in use (0: no list, rebin every step)
    double cell_factor = 1.0;     // triplet cell edge >= cell_factor * rc_triplet
    int lanes = 16;               // lanes per particle in the list force kernel
    int list_cap = 0, pair_cap = 0, nl_cap = 0;  // 0: sized by heuristics
    std::vector<int> tile_need;   // triplet tile entries each system needs (empty: heuristic)
    bool split = false;           // several systems: one triplet launch per tile class
                                  // (systems allowing the same workgroups per CU) instead
                                  // of a single launch at the occupancy of the largest tile
    bool tight = false;           // capacities from observed maxima with thin margins, so
                                  // that the triplet tiles may fit one more workgroup per CU
    bool gather_apart = false;    // F3 summed from the partial slots by its own kernel
                                  // (coalesced, input order) instead of inside the list
                                  // force kernel at x^k (scattered reads, one launch fewer)
};

constexpr int kMaxTileClasses = 8;

// Everything that depends on the configuration: the two cell grids, the capacities and
// the buffers sized by them.  Rebuilt as a whole by build_layout.
struct Layout {
    Config cfg;
    Grid gt, gp;                  // triplet grid, pair grid
    double skin = 0.0;            // == cfg.skin
    int stage_cap = 0, list_cap = 0, pair_cap = 0, nl_cap = 0;  // stage_cap: largest class
    // Tile classes: the triplet cells of systems whose tiles allow the same number of
    // workgroups per CU form one class and one launch, which stages up to cls_cap[c]
    // entries and covers the cells cls_cells[cls_off[c] .. cls_off[c + 1]).
    int ncls = 0;
    int cls_cap[kMaxTileClasses] = {};
    int cls_occ[kMaxTileClasses] = {};  // triplet workgroups per CU of each class
    int cls_off[kMaxTileClasses + 1] = {};
    bool any_whole = false;       // some system's triplet tile is the whole system
    std::vector<int> cls_order;   // host copy of the cell order (all classes)
    int *cls_cells = nullptr;     // [ncell_t] device; nullptr with one class (identity)
    double *ce = nullptr;         // [ncell_t][2] per-cell triplet energy/virial
    long long *cc = nullptr;      // [ncell_t] per-cell triplet counts
    int *nbr = nullptr;           // [n][nl_cap] pair list (pair-grid sorted indices)
};

}  // namespace

// DirectSum mode: the task list of the all-triplets kernel and its partial-force slots.
struct DirectState {
    int ntask = 0, nblk = 0;
    DirectTask *task = nullptr;   // [ntask]
    double *pI = nullptr, *pJ = nullptr, *pK = nullptr;  // partial force slots
    double *ce = nullptr;         // [ntask][2] ATM energy and virial per task
    int *blk_sys = nullptr, *blk0 = nullptr;    // 64-particle blocks (gather)
    int *gslot = nullptr;         // gather sequences of every block (see DirectArgs)
    int64_t *gslot0 = nullptr;    // [nblk + 1]
    SysDesc *sd = nullptr;        // p0, n; cell0/ncell = the system's task range
};

struct mts_system {
    mts_params p{};
    bool direct = false;          // DirectSum: all pairs and triplets, open boundaries
    DirectState dir;
    int nsys = 0;
    int64_t n = 0;
    hipStream_t st = nullptr;
    bool fp32 = false;
    std::vector<SysDesc> base;    // per-system boxes and particle ranges (no grid yet)
    double lmin = 0.0;            // smallest box edge over all systems
    Layout lo;
    size_t max_lds = 64 * 1024;   // per-workgroup LDS limit of the device
    size_t lds_per_cu = 64 * 1024;  // LDS of one CU
    bool collect_stats = false;   // kernels record tile and list maxima into stats
    double tuned_ms = 0.0;        // measured cycle time of the configuration (autotune)
    int tuned_trials = 0;
    double ushift = 0.0;
    std::string err;

    // device buffers (library-owned)
    int *sys_of = nullptr;        // [n]
    int red_chunks = kRedChunks;  // reduction workgroups per system (largest system's count)
    double *red_part = nullptr;   // [nsys][red_chunks][6] reduction partials
    int *red_done = nullptr;      // [nsys + 1] reduction completion counters (zero at rest)
    double *f2a = nullptr, *f2b = nullptr, *f3 = nullptr;  // [n][3] force caches
    double *pf = nullptr;         // [14][3][n] triplet partial slots
    int k2 = 1;                   // nested r-RESPA: mid cycles per full step (k_outer, >= 1)
    double *pe = nullptr;         // [n][2] per-particle pair energy/virial (pair-grid order)
    long long *cnt_sys = nullptr; // [nsys]
    int *nn = nullptr;            // [n]
    int *stats = nullptr;         // [4] observed maxima (tile and list sizes), tuning only
    int *tile_obs = nullptr;      // [nsys] largest triplet tile seen per system (overflow,
                                  // tuning), zeroed after reading
    double *x_ref = nullptr;      // [n][3] wrapped positions at the last list build (pair grid order)
    int *flags = nullptr;
    int *row = nullptr;
    double *e_buf = nullptr;      // [e_rows][nsys][5] energy records of one respa_step
    int64_t e_rows = 0;
    unsigned long long *list_n = nullptr;

    // r-RESPA cycles run on an internal stream, optionally replayed from captured graphs
    hipStream_t ist = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    bool use_graph = true;
    // [energies][F2 parity][ends a full step][continues a call: opening done by the last]
    hipGraphExec_t gexec[2][2][2][2] = {};
    double *xi = nullptr, *vi = nullptr;  // internal copies of x and v, [n][3]
    // v and two F2 caches in the pair grid's sorted order, for the inner steps between
    // the first and the last of a cycle with a pair list
    double *vs = nullptr, *f2s[2] = {nullptr, nullptr};

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

#define HIP_TRY(sys, expr)                                     \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return hip_fail(sys, _e, #expr); \
    } while (0)

#define MTS_TRY(expr)                \
    do {                             \
        mts_status _r = (expr);      \
        if (_r != MTS_OK) return _r; \
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
    if (!std::isfinite(p->skin) || p->skin < 0.0) { msg = "skin must be finite and >= 0"; return MTS_ERR_INVALID_ARG; }
    if (p->k < 1) { msg = "k (step-size factor) must be >= 1"; return MTS_ERR_INVALID_ARG; }
    if (p->precision != MTS_FP64 && p->precision != MTS_FP32) { msg = "unknown precision"; return MTS_ERR_INVALID_ARG; }
    if (p->method != MTS_CUTOFF && p->method != MTS_DIRECT) { msg = "unknown method"; return MTS_ERR_INVALID_ARG; }
    if (p->k_outer < 0) { msg = "k_outer must be >= 0"; return MTS_ERR_INVALID_ARG; }
    if (p->k_outer > 1) {
        if (!(p->rc_triplet_inner > 0.0 && p->rc_triplet_inner < p->rc_triplet)) {
            msg = "rc_triplet_inner must lie in (0, rc_triplet) when k_outer > 1";
            return MTS_ERR_INVALID_ARG;
        }
        if (p->method == MTS_DIRECT) {
            msg = "triplet distance classes need the cutoff method";
            return MTS_ERR_UNSUPPORTED;
        }
    } else if (p->rc_triplet_inner != 0.0) {
        msg = "rc_triplet_inner must be 0 unless k_outer > 1";
        return MTS_ERR_INVALID_ARG;
    }
    return MTS_OK;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Grid with cell edges of at least hmin (margin against rounding so that any pair within
// the cutoff lies in adjacent cells), at least 2 cells per edge.
mts_status make_grid(Grid &g, const std::vector<SysDesc> &base, double hmin, bool triplet) {
    g.hsd = base;
    int64_t cell0 = 0;
    for (SysDesc &d : g.hsd) {
        for (int k = 0; k < 3; ++k) {
            d.nc[k] = (int)std::floor(d.L[k] / hmin);
            if (d.nc[k] < 2) return MTS_ERR_BOX_TOO_SMALL;
            d.q[k] = (double)d.nc[k] / d.L[k];
        }
        d.ncell = d.nc[0] * d.nc[1] * d.nc[2];
        d.whole = triplet && d.ncell < kNumHalf ? 1 : 0;
        d.cell0 = (int)cell0;
        cell0 += d.ncell;
    }
    if (cell0 >= (int64_t)1 << 30) return MTS_ERR_UNSUPPORTED;
    g.ncell = (int)cell0;
    return MTS_OK;
}

double max_cell_volume(const Grid &g, double &rho_max) {
    double v = 0.0;
    rho_max = 0.0;
    for (const SysDesc &d : g.hsd) {
        const double vol = d.L[0] * d.L[1] * d.L[2];
        const double rho = std::max(0.9, 1.2 * (double)d.n / vol);
        rho_max = std::max(rho_max, rho);
        v = std::max(v, rho * (d.L[0] / d.nc[0]) * (d.L[1] / d.nc[1]) * (d.L[2] / d.nc[2]));
    }
    return v;
}

// The triplet kernel's hit queue stores list positions in 8 bits.
constexpr int kMaxListCap = 256;

// Tile and list capacities.  A cell of volume h^3 holds about rho h^3 particles; sizing
// assumes a local density of max(0.9, 1.2 x the system's mean), which covers LJ liquids
// and crystals near the densities of the paper's scenarios, including a liquid slab
// inside a dilute box.  The triplet tile holds the 14 cells of the forward half stencil
// and the pair tile all 27 cells of the pair grid.  An anchor's forward-neighbour list
// holds half a cutoff sphere on average but, for an anchor at the low corner of its cell,
// up to about a whole one, so it is sized like a pair-list row (a whole (rc + skin)
// sphere).  Overflow is
// detected on the device, reported by mts_sync, and doubles the capacity for the next
// call; mts_autotune sizes them from the maxima observed on the real input instead.
void size_tiles(const mts_system *s, Layout &lo) {
    double rho_t, rho_p;
    (void)max_cell_volume(lo.gt, rho_t);
    const double vp = max_cell_volume(lo.gp, rho_p);
    const double rc3 = s->p.rc_triplet, rv = s->p.rc_pair + lo.skin;
    lo.cfg.tile_need.resize(s->nsys);
    for (int q = 0; q < s->nsys; ++q) {
        const SysDesc &d = lo.gt.hsd[q];
        const double rho = std::max(0.9, 1.2 * (double)d.n / (d.L[0] * d.L[1] * d.L[2]));
        const double v = rho * (d.L[0] / d.nc[0]) * (d.L[1] / d.nc[1]) * (d.L[2] / d.nc[2]);
        // a whole-system tile holds exactly the system's particles
        lo.cfg.tile_need[q] = d.whole ? (int)d.n : (int)std::ceil(kNumHalf * v * 1.1) + 16;
    }
    lo.pair_cap = std::min(2048, round_up((int)std::ceil(kNumFull * vp * 1.1) + 16, 32));
    lo.list_cap = std::min(kMaxListCap, round_up((int)std::ceil(1.25 * rho_t * (4.0 / 3.0) * M_PI * rc3 * rc3 * rc3) + 8, 16));
    lo.nl_cap = std::min(2048, round_up((int)std::ceil(1.3 * rho_p * (4.0 / 3.0) * M_PI * rv * rv * rv) + 16, 32));
}

mts_status alloc_grid(mts_system *s, Grid &g) {
    const int64_t n = s->n;
    HIP_TRY(s, dalloc(&g.sd, s->nsys));
    HIP_TRY(s, dalloc(&g.sys_of_cell, g.ncell));
    HIP_TRY(s, dalloc(&g.cell_of, n));
    HIP_TRY(s, dalloc(&g.rank, n));
    HIP_TRY(s, dalloc(&g.count, g.ncell));
    HIP_TRY(s, dalloc(&g.start, (size_t)g.ncell + 1));
    const size_t ntile = ((size_t)g.ncell + kScanTile - 1) / kScanTile;
    HIP_TRY(s, dalloc(&g.start_loc, (size_t)g.ncell));
    HIP_TRY(s, dalloc(&g.tile_sum, 2 * ntile + 1));
    HIP_TRY(s, hipMemset(g.tile_sum, 0, sizeof(int) * (2 * ntile + 1)));
    HIP_TRY(s, dalloc(&g.perm_tmp, n));
    HIP_TRY(s, dalloc(&g.perm, n));
    HIP_TRY(s, dalloc(&g.inv_perm, n));
    HIP_TRY(s, dalloc(&g.xs, n));
    HIP_TRY(s, dalloc(&g.xs2, n));
    std::vector<int> soc(g.ncell);
    for (int q = 0; q < s->nsys; ++q) {
        const SysDesc &d = g.hsd[q];
        for (int c = 0; c < d.ncell; ++c) soc[d.cell0 + c] = q;
    }
    HIP_TRY(s, hipMemcpy(g.sd, g.hsd.data(), sizeof(SysDesc) * s->nsys, hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(g.sys_of_cell, soc.data(), sizeof(int) * g.ncell, hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemset(g.count, 0, sizeof(int) * g.ncell));
    return MTS_OK;
}

void free_grid(Grid &g) {
    void *ptrs[] = {g.sd, g.sys_of_cell, g.cell_of, g.rank, g.count, g.start, g.start_loc, g.tile_sum, g.perm_tmp,
                    g.perm, g.inv_perm, g.xs, g.xs2};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    g = Grid{};
}

void free_layout(Layout &lo) {
    free_grid(lo.gt);
    free_grid(lo.gp);
    void *ptrs[] = {lo.ce, lo.cc, lo.nbr, lo.cls_cells};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    lo = Layout{};
}

// Cells are strictly wider than the cutoff, with margin for rounding, so that any
// interacting pair lies in adjacent cells.
constexpr double kCellMargin = 1.0 + 1e-9;

// The pair-list skin actually used for a requested one: shrunk so that every box edge
// exceeds 2 (rc + skin) -- a pair then has one image within the list radius -- and
// dropped (no list; every step rebins) below 0.05 sigma, where a list does not pay.
double effective_skin(const mts_system *s, double skin) {
    skin = std::min(skin, 0.4999 * s->lmin / kCellMargin - s->p.rc_pair);
    return skin >= 0.05 * s->p.sigma ? skin : 0.0;
}

// Largest tile capacity (a multiple of 32) whose triplet workgroup fits `limit` bytes of
// LDS with lists of lc entries.
int cap_for_lds(const mts_system *s, int lc, size_t limit) {
    int lo = 0, hi = 4096 / 32;  // in units of 32 entries
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (triplet_lds_bytes(32 * mid, lc, s->fp32) <= limit) lo = mid;
        else hi = mid - 1;
    }
    return 32 * lo;
}

// The triplet launches of a force evaluation.  By default one launch (a single tile
// class): its tile capacity is the largest need of any system, raised to the largest
// capacity that keeps the same number of workgroups per CU (headroom against overflow at
// no cost in occupancy).  With cfg.split (a tuning choice for batches) the systems are
// grouped into tile classes by the workgroups per CU their tiles allow, one launch per
// class, so that a few large tiles do not set the occupancy of the whole batch.  Within a
// launch the base cells of several systems are ordered by decreasing estimated work per
// cell (anchors per cell x tile entries), so that the dispatcher starts the costly items
// first.  Whole-system tiles (boxes of fewer than 14 cells) hold N entries instead of 14
// cells' worth.
mts_status classify(const mts_system *s, Layout &lo) {
    const int lc = lo.list_cap;
    lo.any_whole = false;
    for (const SysDesc &d : lo.gt.hsd) lo.any_whole = lo.any_whole || d.whole;
    const int cmax = cap_for_lds(s, lc, s->max_lds);
    auto occ = [&](int cap) {
        const size_t b = triplet_lds_bytes(cap, lc, s->fp32);
        const int r = triplet_blocks_per_cu(s->fp32, lo.any_whole, b, s->lds_per_cu);
        return r > 0 ? r : std::max(1, std::min(2, (int)(s->lds_per_cu / (b + 2048))));
    };
    std::vector<int> occ_of(s->nsys), level;
    int need_max = 32;
    for (int q = 0; q < s->nsys; ++q) {
        const int c = round_up(std::max(32, lo.cfg.tile_need[q]), 32);
        if (c > cmax) return MTS_ERR_UNSUPPORTED;
        need_max = std::max(need_max, c);
        occ_of[q] = lo.cfg.split ? occ(c) : 0;
        if (std::find(level.begin(), level.end(), occ_of[q]) == level.end()) level.push_back(occ_of[q]);
    }
    if (!lo.cfg.split) level.assign(1, occ(need_max));
    if ((int)level.size() > kMaxTileClasses) return MTS_ERR_UNSUPPORTED;
    std::sort(level.begin(), level.end(), [](int a, int b) { return a > b; });
    // estimated work per cell of each system, for the order of the cells
    std::vector<std::pair<double, int>> work(s->nsys);
    for (int q = 0; q < s->nsys; ++q) {
        const SysDesc &d = lo.gt.hsd[q];
        const double per_cell = (double)d.n / std::max(1, d.ncell);
        work[q] = {-per_cell * (d.whole ? (double)d.n : kNumHalf * per_cell), q};
    }
    std::stable_sort(work.begin(), work.end());
    lo.ncls = (int)level.size();
    lo.stage_cap = 0;
    lo.cls_order.clear();
    for (int c = 0; c < lo.ncls; ++c) {
        const bool in_class_all = !lo.cfg.split;
        int lo_i = 1;
        for (int q = 0; q < s->nsys; ++q)
            if (in_class_all || occ_of[q] == level[c])
                lo_i = std::max(lo_i, round_up(std::max(32, lo.cfg.tile_need[q]), 32) / 32);
        int hi_i = cmax / 32;
        while (lo_i < hi_i) {  // largest capacity with at least this occupancy
            const int mid = (lo_i + hi_i + 1) / 2;
            if (occ(32 * mid) >= level[c]) lo_i = mid;
            else hi_i = mid - 1;
        }
        lo.cls_cap[c] = 32 * lo_i;
        lo.cls_occ[c] = occ(lo.cls_cap[c]);
        lo.stage_cap = std::max(lo.stage_cap, lo.cls_cap[c]);
        lo.cls_off[c] = (int)lo.cls_order.size();
        for (const auto &w : work)
            if (in_class_all || occ_of[w.second] == level[c]) {
                const SysDesc &d = lo.gt.hsd[w.second];
                for (int k = 0; k < d.ncell; ++k) lo.cls_order.push_back(d.cell0 + k);
            }
    }
    lo.cls_off[lo.ncls] = (int)lo.cls_order.size();
    if (s->nsys == 1) lo.cls_order.clear();  // identity order, no cell map
    return MTS_OK;
}

// The cell order on the device (none for a single system: identity order).
mts_status upload_classes(mts_system *s, Layout &lo) {
    if (lo.cls_order.empty()) return MTS_OK;
    if (!lo.cls_cells) HIP_TRY(s, dalloc(&lo.cls_cells, lo.gt.ncell));
    HIP_TRY(s, hipMemcpy(lo.cls_cells, lo.cls_order.data(), sizeof(int) * lo.cls_order.size(),
                         hipMemcpyHostToDevice));
    return MTS_OK;
}

// Builds a complete layout for cfg into `out` without touching the handle's own.
mts_status build_layout(mts_system *s, const Config &cfg, Layout &out) {
    out = Layout{};
    out.cfg = cfg;
    out.skin = cfg.skin;
    mts_status r = make_grid(out.gt, s->base, cfg.cell_factor * s->p.rc_triplet * kCellMargin, true);
    if (r == MTS_OK) r = make_grid(out.gp, s->base, (s->p.rc_pair + cfg.skin) * kCellMargin, false);
    if (r != MTS_OK) {
        out = Layout{};
        return r;
    }
    size_tiles(s, out);
    if ((int)cfg.tile_need.size() == s->nsys) out.cfg.tile_need = cfg.tile_need;
    if (cfg.list_cap > 0) out.list_cap = cfg.list_cap;
    if (cfg.pair_cap > 0) out.pair_cap = cfg.pair_cap;
    if (cfg.nl_cap > 0) out.nl_cap = cfg.nl_cap;
    out.cfg.list_cap = out.list_cap;
    out.cfg.pair_cap = out.pair_cap;
    out.cfg.nl_cap = out.nl_cap;
    if (classify(s, out) != MTS_OK || pair_lds_bytes(out.pair_cap) > s->max_lds) {
        out = Layout{};
        return MTS_ERR_UNSUPPORTED;
    }
    r = alloc_grid(s, out.gt);
    if (r == MTS_OK) r = alloc_grid(s, out.gp);
    if (r == MTS_OK) r = upload_classes(s, out);
    if (r == MTS_OK && (dalloc(&out.ce, 2 * (size_t)out.gt.ncell) != hipSuccess ||
                        dalloc(&out.cc, out.gt.ncell) != hipSuccess ||
                        dalloc(&out.nbr, (size_t)s->n * out.nl_cap) != hipSuccess ||
                        hipMemset(out.ce, 0, 2 * sizeof(double) * out.gt.ncell) != hipSuccess))
        r = fail(s, MTS_ERR_OOM, "device memory for the cell grids and lists");
    if (r != MTS_OK) {
        free_layout(out);
        return r == MTS_ERR_HIP ? MTS_ERR_OOM : r;
    }
    return MTS_OK;
}

// Buffers that depend on the particle and system counts only.
mts_status alloc_all(mts_system *s) {
    const int64_t n = s->n;
    HIP_TRY(s, dalloc(&s->sys_of, n));
    s->red_chunks = kRedChunks;
    for (const SysDesc &d : s->base) s->red_chunks = std::max(s->red_chunks, red_chunks(d.n));
    HIP_TRY(s, dalloc(&s->red_part, (size_t)s->nsys * s->red_chunks * 6));
    HIP_TRY(s, dalloc(&s->red_done, (size_t)s->nsys + 1));
    HIP_TRY(s, hipMemset(s->red_done, 0, sizeof(int) * (s->nsys + 1)));
    HIP_TRY(s, dalloc(&s->f2a, 3 * n));
    HIP_TRY(s, dalloc(&s->f2b, 3 * n));
    HIP_TRY(s, dalloc(&s->f3, 3 * n));
    HIP_TRY(s, dalloc(&s->pf, (size_t)kNumHalf * 3 * n));
    HIP_TRY(s, dalloc(&s->pe, 2 * n));
    HIP_TRY(s, dalloc(&s->cnt_sys, s->nsys));
    HIP_TRY(s, dalloc(&s->nn, n));
    HIP_TRY(s, dalloc(&s->stats, 4));
    HIP_TRY(s, dalloc(&s->tile_obs, s->nsys));
    HIP_TRY(s, hipMemset(s->tile_obs, 0, sizeof(int) * s->nsys));
    HIP_TRY(s, dalloc(&s->x_ref, 3 * n));
    HIP_TRY(s, dalloc(&s->flags, 1));
    HIP_TRY(s, dalloc(&s->row, 2));
    HIP_TRY(s, dalloc(&s->list_n, 1));
    HIP_TRY(s, dalloc(&s->xi, 3 * n));
    HIP_TRY(s, dalloc(&s->vi, 3 * n));
    if (!s->direct) {
        HIP_TRY(s, dalloc(&s->vs, 3 * n));
        HIP_TRY(s, dalloc(&s->f2s[0], 3 * n));
        HIP_TRY(s, dalloc(&s->f2s[1], 3 * n));
    }
    HIP_TRY(s, hipStreamCreateWithFlags(&s->ist, hipStreamNonBlocking));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));

    std::vector<int> so(n > 0 ? n : 1);
    for (int q = 0; q < s->nsys; ++q) {
        const SysDesc &d = s->base[q];
        for (int64_t i = 0; i < d.n; ++i) so[d.p0 + i] = q;
    }
    if (n > 0) HIP_TRY(s, hipMemcpy(s->sys_of, so.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemset(s->flags, 0, sizeof(int)));
    if (n > 0) HIP_TRY(s, hipMemset(s->pf, 0, sizeof(double) * kNumHalf * 3 * n));
    return MTS_OK;
}

void drop_graphs(mts_system *s) {
    for (auto &g : s->gexec)
        for (auto &h : g)
            for (auto &i : h)
                for (hipGraphExec_t &e : i)
                    if (e) {
                        (void)hipGraphExecDestroy(e);
                        e = nullptr;
                    }
}

// Replaces the handle's layout by one built for cfg (the old one stays on failure).
mts_status set_layout(mts_system *s, const Config &cfg) {
    Layout nl;
    MTS_TRY(build_layout(s, cfg, nl));
    if (s->ist) (void)hipStreamSynchronize(s->ist);
    (void)hipStreamSynchronize(s->st);
    drop_graphs(s);  // captured launches carry the old buffers and sizes
    free_layout(s->lo);
    s->lo = nl;
    return MTS_OK;
}

void free_direct(DirectState &d) {
    void *ptrs[] = {d.task, d.pI, d.pJ, d.pK, d.ce, d.blk_sys, d.blk0, d.gslot, d.gslot0, d.sd};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = DirectState{};
}

// DirectSum set-up: per system, the block triples (I <= J <= K) of 64-particle blocks
// (split along j into up to kDirMaxSplit tasks for small systems), and for the gather
// kernel the block table and each block's sequence of slots.
mts_status setup_direct(mts_system *s) {
    DirectState &D = s->dir;
    std::vector<DirectTask> tasks;
    std::vector<int> blk_sys, blk0(s->nsys), task_of;
    std::vector<int64_t> task_of0(s->nsys), gslot0;
    std::vector<int> gslot;
    std::vector<SysDesc> sd = s->base;
    for (int q = 0; q < s->nsys; ++q) {
        const int n = (int)s->base[q].n;
        const int nb = (n + kDirBlock - 1) / kDirBlock;
        // split the j range of each triple so that the system alone makes ~kDirTaskTarget
        // tasks (a power of two, at most kDirMaxSplit, so that 64 / split >= 8 j per task)
        const int64_t triples = (int64_t)nb * (nb + 1) * (nb + 2) / 6;
        int sp = 1;
        while (sp < kDirMaxSplit && triples > 0 && triples * sp < kDirTaskTarget) sp *= 2;
        sd[q].cell0 = (int)tasks.size();
        task_of0[q] = (int64_t)task_of.size();
        task_of.resize(task_of.size() + (size_t)nb * nb * nb, -1);
        for (int I = 0; I < nb; ++I)
            for (int J = I; J < nb; ++J)
                for (int K = J; K < nb; ++K) {
                    task_of[task_of0[q] + ((int64_t)I * nb + J) * nb + K] = (int)tasks.size();
                    for (int u = 0; u < sp; ++u)
                        tasks.push_back(DirectTask{q, I, J, K, u * (kDirBlock / sp),
                                                   (u + 1) * (kDirBlock / sp)});
                }
        sd[q].ncell = (int)tasks.size() - sd[q].cell0;
        blk0[q] = (int)blk_sys.size();
        for (int b = 0; b < nb; ++b) blk_sys.push_back(q);
        // gather sequence of block X: its slots as I, then as J, then as K
        auto tof = [&](int I, int J, int K) {
            return task_of[task_of0[q] + ((int64_t)I * nb + J) * nb + K];
        };
        for (int X = 0; X < nb; ++X) {
            gslot0.push_back((int64_t)gslot.size());
            auto push = [&](int role, int first) {
                for (int u = 0; u < sp; ++u) gslot.push_back((role << 30) | (first + u));
            };
            for (int J = X; J < nb; ++J)
                for (int K = J; K < nb; ++K) push(0, tof(X, J, K));
            for (int I = 0; I <= X; ++I)
                for (int K = X; K < nb; ++K) push(1, tof(I, X, K));
            for (int J = 0; J <= X; ++J)
                for (int I = 0; I <= J; ++I) push(2, tof(I, J, X));
        }
    }
    gslot0.push_back((int64_t)gslot.size());
    if (tasks.size() >= (size_t)1 << 30)  // task indices carry a 2-bit role in gslot
        return fail(s, MTS_ERR_UNSUPPORTED, "too many particles for DirectSum");
    D.ntask = (int)tasks.size();
    D.nblk = (int)blk_sys.size();
    const size_t slot = 3 * kDirBlock;
    HIP_TRY(s, dalloc(&D.task, tasks.size()));
    HIP_TRY(s, dalloc(&D.pI, tasks.size() * slot));
    HIP_TRY(s, dalloc(&D.pJ, tasks.size() * slot));
    HIP_TRY(s, dalloc(&D.pK, tasks.size() * slot));
    HIP_TRY(s, dalloc(&D.ce, 2 * tasks.size()));
    HIP_TRY(s, dalloc(&D.blk_sys, blk_sys.size()));
    HIP_TRY(s, dalloc(&D.blk0, blk0.size()));
    HIP_TRY(s, dalloc(&D.gslot, gslot.size()));
    HIP_TRY(s, dalloc(&D.gslot0, gslot0.size()));
    HIP_TRY(s, dalloc(&D.sd, sd.size()));
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    HIP_TRY(s, up(D.task, tasks.data(), sizeof(DirectTask) * tasks.size()));
    HIP_TRY(s, up(D.blk_sys, blk_sys.data(), sizeof(int) * blk_sys.size()));
    HIP_TRY(s, up(D.blk0, blk0.data(), sizeof(int) * blk0.size()));
    HIP_TRY(s, up(D.gslot, gslot.data(), sizeof(int) * gslot.size()));
    HIP_TRY(s, up(D.gslot0, gslot0.data(), sizeof(int64_t) * gslot0.size()));
    HIP_TRY(s, up(D.sd, sd.data(), sizeof(SysDesc) * sd.size()));
    if (!tasks.empty()) HIP_TRY(s, hipMemset(D.ce, 0, sizeof(double) * 2 * tasks.size()));
    return MTS_OK;
}

void free_all(mts_system *s) {
    free_direct(s->dir);
    drop_graphs(s);
    if (s->ev_in) (void)hipEventDestroy(s->ev_in);
    if (s->ev_out) (void)hipEventDestroy(s->ev_out);
    if (s->ist) (void)hipStreamDestroy(s->ist);
    for (int c = 0; c < 2; ++c)
        for (hipEvent_t e : s->ev_pool[c]) (void)hipEventDestroy(e);
    free_layout(s->lo);
    void *ptrs[] = {s->sys_of, s->red_part, s->red_done, s->f2a, s->f2b, s->f3, s->pf, s->pe, s->cnt_sys,
                    s->nn, s->stats, s->tile_obs, s->x_ref, s->flags, s->row, s->e_buf, s->list_n,
                    s->xi, s->vi, s->vs, s->f2s[0], s->f2s[1]};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
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

// ---- enqueue helpers (all on s->st)

enum : int { kBinPair = 1, kBinTriplet = 2 };

void fill_bin_grid(BinGrid &b, Grid &g, double *x_ref) {
    b.sd = g.sd;
    b.ncell = g.ncell;
    b.cell_of = g.cell_of;
    b.rank = g.rank;
    b.count = g.count;
    b.start = g.start;
    b.start_loc = g.start_loc;
    b.tile_sum = g.tile_sum;
    b.tmp = g.perm_tmp;
    b.perm = g.perm;
    b.inv_perm = g.inv_perm;
    b.xs = g.xs;
    b.x_ref = x_ref;
}

// Counting sort of x into the pair grid and/or the triplet grid (one launch per pass);
// with_ref also records the wrapped positions as the reference of the next skin check.
mts_status enqueue_bin(mts_system *s, int which, const double *x, bool with_ref) {
    BinArgs a{};
    a.n = s->n;
    a.x = x;
    a.sys_of = s->sys_of;
    a.flags = s->flags;
    if (which & kBinPair) fill_bin_grid(a.g[a.ng++], s->lo.gp, with_ref ? s->x_ref : nullptr);
    if (which & kBinTriplet) fill_bin_grid(a.g[a.ng++], s->lo.gt, nullptr);
    HIP_TRY(s, launch_bin(s->st, a));
    return MTS_OK;
}

// F2 from the pair grid's cell tiles (no list).
mts_status enqueue_pair(mts_system *s, double *f2) {
    const Grid &g = s->lo.gp;
    PairArgs a{};
    a.ncell = g.ncell;
    a.sys_of_cell = g.sys_of_cell;
    a.stage_cap = s->lo.pair_cap;
    a.n = s->n;
    a.xs = g.xs;
    a.perm = g.perm;
    a.start = g.start;
    a.sd = g.sd;
    a.sys_of = s->sys_of;
    a.f = f2;
    a.pe = s->pe;
    a.eps = s->p.epsilon;
    a.sigma2 = s->p.sigma * s->p.sigma;
    a.rc2 = s->p.rc_pair * s->p.rc_pair;
    a.ushift = s->ushift;
    a.flags = s->flags;
    const long ts = timer_begin(s, 1);
    HIP_TRY(s, launch_pair(s->st, a));
    timer_end(s, 1, ts);
    return MTS_OK;
}

// Verlet list of the pair grid at its current binning.
ListBuildArgs list_build_args(const mts_system *s) {
    const Grid &g = s->lo.gp;
    ListBuildArgs a{};
    a.ncell = g.ncell;
    a.sys_of_cell = g.sys_of_cell;
    a.stage_cap = s->lo.pair_cap;
    a.n = s->n;
    a.xs = g.xs;
    a.start = g.start;
    a.sd = g.sd;
    a.nbr = s->lo.nbr;
    a.nn = s->nn;
    a.nl_cap = s->lo.nl_cap;
    const double rv = s->p.rc_pair + s->lo.skin;
    a.rv2 = rv * rv;
    a.flags = s->flags;
    a.stats = s->collect_stats ? s->stats + 2 : nullptr;
    return a;
}

mts_status enqueue_list_build(mts_system *s) {
    HIP_TRY(s, launch_list_build(s->st, list_build_args(s)));
    return MTS_OK;
}

// Update steps fused behind the list forces (see PairListArgs).
// Which triplet forces an evaluation leaves in the slots pf.  Without distance classes
// (k_outer = 1, and every standalone call) those of T(rc3).  Nested r-RESPA: at a full step
// the weighted pass over T(rc3), F_in + k_outer F_out (the two kicks that fall together
// there, both applied with dt k / 2m); between full steps the inner class alone.
enum F3Mode { kF3All, kF3Outer, kF3Inner };

F3Mode cycle_mode(const mts_system *s, bool full) {
    return s->k2 == 1 ? kF3All : (full ? kF3Outer : kF3Inner);
}

struct Fused {
    bool kick2 = false, kick3_end = false, kick3_start = false, drift = false;
    bool gather3 = false;  // gather F3 from the partial slots (into s->f3) first
    // v and the previous F2 read in the pair grid's sorted order (s->vs), F2 and v
    // written in it (and x not written); see PairListArgs
    bool in_sorted = false, out_sorted = false;
    // also the next cycle's opening (F3 half kick, first drift) into s->vs, s->f2s[0] and
    // the pair grid's second position buffer; see PairListArgs
    bool open_next = false;
    const double *f2prev = nullptr;
    Pos4 *xs_out = nullptr;
};

// F2 from the pair list at positions xs_in (pair grid sorted order) into f2, then the
// fused update u of the internal x, v (u.drift writes the new positions to u.xs_out).
mts_status enqueue_pair_list(mts_system *s, const Pos4 *xs_in, double *f2, const Fused &u,
                             bool energy) {
    const double dt = s->p.dt, m = s->p.mass;
    PairListArgs a{};
    a.n = s->n;
    a.xs = xs_in;
    a.perm = s->lo.gp.perm;
    a.lanes = s->lo.cfg.lanes;
    a.nbr = s->lo.nbr;
    a.nn = s->nn;
    a.nl_cap = s->lo.nl_cap;
    a.sd = s->lo.gp.sd;
    a.sys_of = s->sys_of;
    a.f = f2;
    a.pe = energy ? s->pe : nullptr;
    a.eps = s->p.epsilon;
    a.sigma2 = s->p.sigma * s->p.sigma;
    a.rc2 = s->p.rc_pair * s->p.rc_pair;
    a.ushift = s->ushift;
    a.flags = s->flags;
    if (u.gather3) {
        a.pf = s->pf;
        a.inv_perm3 = s->lo.gt.inv_perm;
        a.f3_out = s->f3;
    }
    if (u.kick2 || u.kick3_end || u.kick3_start || u.drift) {
        a.kick2 = u.kick2;
        a.kick3_end = u.kick3_end;
        a.kick3_start = u.kick3_start;
        a.drift = u.drift;
        a.in_sorted = u.in_sorted;
        a.out_sorted = u.out_sorted;
        a.x = u.out_sorted ? nullptr : s->xi;
        a.v_in = u.in_sorted ? s->vs : s->vi;
        a.v_out = u.out_sorted ? s->vs : s->vi;
        a.f2prev = u.f2prev;
        a.f3 = s->f3;
        a.c2 = dt / (2.0 * m);
        a.c3 = (dt * (double)s->p.k) / (2.0 * m);
        a.dt = dt;
        a.cx = (dt * dt) / (2.0 * m);
        a.xs_out = u.xs_out;
        a.x_ref = (u.drift && u.xs_out) || u.open_next ? s->x_ref : nullptr;
        if (u.open_next) {
            a.open_next = 1;
            a.v_next = s->vs;
            a.f2_next = s->f2s[0];
            a.xs_next = s->lo.gp.xs2;
        }
        a.half_skin2 = 0.25 * s->lo.skin * s->lo.skin;
    }
    const long ts = timer_begin(s, 1);
    HIP_TRY(s, launch_pair_list(s->st, a));
    timer_end(s, 1, ts);
    return MTS_OK;
}

// Arguments of the launch of tile class cls for mode: kF3Inner evaluates the inner
// distance class (all edges <= rc_triplet_inner), without energies or counts; kF3Outer
// weights the outer class's forces by k_outer.
TripletArgs triplet_args(const mts_system *s, int cls, int *list_ijk, long long list_rows,
                         bool energy, F3Mode mode = kF3All) {
    const Layout &lo = s->lo;
    const Grid &g = lo.gt;
    TripletArgs a{};
    a.ncell = lo.cls_off[cls + 1] - lo.cls_off[cls];
    a.cell_map = lo.cls_cells ? lo.cls_cells + lo.cls_off[cls] : nullptr;
    a.any_whole = lo.any_whole ? 1 : 0;
    a.xs = g.xs;
    a.start = g.start;
    a.sd = g.sd;
    a.sys_of_cell = g.sys_of_cell;
    a.perm = g.perm;
    a.pf = s->pf;
    a.ce = energy ? s->lo.ce : nullptr;
    a.cc = s->lo.cc;
    a.n = s->n;
    a.nu = s->p.nu;
    a.rc2 = s->p.rc_triplet * s->p.rc_triplet;
    a.stage_cap = lo.cls_cap[cls];
    a.occ6 = lo.cls_occ[cls] >= 6 ? 1 : 0;
    a.list_cap = lo.list_cap;
    a.flags = s->flags;
    a.list_ijk = list_ijk;
    a.list_n = s->list_n;
    a.list_rows = list_rows;
    a.stats = s->collect_stats ? s->stats : nullptr;
    a.tile_obs = s->tile_obs;
    if (mode == kF3Inner) {
        a.rc2 = s->p.rc_triplet_inner * s->p.rc_triplet_inner;
        a.ce = nullptr;
        a.cc = nullptr;
        a.stats = nullptr;
        a.list_ijk = nullptr;
    } else if (mode == kF3Outer) {
        a.ra2 = s->p.rc_triplet_inner * s->p.rc_triplet_inner;
        a.w_out = (double)s->k2;
        a.list_ijk = nullptr;
    }
    return a;
}

// The triplet partial slots of every cell for mode (one launch per tile class and
// class of triplets), then, when f3 is given, their gather into f3.
mts_status enqueue_triplet(mts_system *s, double *f3, int *list_ijk, long long list_rows,
                           bool energy, F3Mode mode = kF3All) {
    const long ts = timer_begin(s, 0);
    for (int c = 0; c < s->lo.ncls; ++c)
        HIP_TRY(s, launch_triplet(s->st, triplet_args(s, c, list_ijk, list_rows, energy, mode),
                                  s->fp32, list_ijk != nullptr));
    timer_end(s, 0, ts);
    if (f3) HIP_TRY(s, launch_triplet_gather(s->st, s->n, s->pf, s->lo.gt.perm, f3, s->flags));
    return MTS_OK;
}

// The triplet partial slots for mode and the new pair list: the list build shares the
// launch of the first tile class (timed together as kernel class 0).
mts_status enqueue_triplet_and_list(mts_system *s, bool energy, F3Mode mode) {
    const long ts = timer_begin(s, 0);
    HIP_TRY(s, launch_triplet_and_list(s->st, triplet_args(s, 0, nullptr, 0, energy, mode),
                                       list_build_args(s), s->fp32));
    for (int c = 1; c < s->lo.ncls; ++c)
        HIP_TRY(s, launch_triplet(s->st, triplet_args(s, c, nullptr, 0, energy, mode), s->fp32,
                                  false));
    timer_end(s, 0, ts);
    return MTS_OK;
}

// DirectSum pair forces at x into f2 (halved pair energies into pe when asked for), timed
// as kernel class 1.
mts_status enqueue_direct_pair(mts_system *s, const double *x, double *f2, bool energy) {
    DirectPairArgs a{};
    a.n = s->n;
    a.sys_of = s->sys_of;
    a.sd = s->dir.sd;
    a.x = x;
    a.f = f2;
    a.pe = energy ? s->pe : nullptr;
    a.eps = s->p.epsilon;
    a.sigma2 = s->p.sigma * s->p.sigma;
    a.flags = s->flags;
    const long ts = timer_begin(s, 1);
    HIP_TRY(s, launch_direct_pair(s->st, a));
    timer_end(s, 1, ts);
    return MTS_OK;
}

// DirectSum triplet forces at x into f3 (per-task energies when asked for); the triplet
// kernel is timed as kernel class 0, the gather is not.
mts_status enqueue_direct_triplet(mts_system *s, const double *x, double *f3, bool energy) {
    const DirectState &D = s->dir;
    DirectArgs a{};
    a.ntask = D.ntask;
    a.task = D.task;
    a.sd = D.sd;
    a.x = x;
    a.nu = s->p.nu;
    a.pI = D.pI;
    a.pJ = D.pJ;
    a.pK = D.pK;
    a.ce = D.ce;
    a.nblk = D.nblk;
    a.blk_sys = D.blk_sys;
    a.blk0 = D.blk0;
    a.gslot = D.gslot;
    a.gslot0 = D.gslot0;
    a.flags = s->flags;
    const long ts = timer_begin(s, 0);
    HIP_TRY(s, launch_direct_triplet(s->st, a, s->fp32, energy));
    timer_end(s, 0, ts);
    HIP_TRY(s, launch_direct_gather(s->st, a, f3));
    return MTS_OK;
}

mts_status enqueue_reduce(mts_system *s, const double *v, bool pair, bool trip, double *out,
                          int stride, int *row, long long *count_out) {
    ReduceArgs a{};
    a.nsys = s->nsys;
    a.sd = s->direct ? s->dir.sd : s->lo.gt.sd;  // direct: "cells" are the triplet tasks
    a.v = v;
    a.half_mass = 0.5 * s->p.mass;
    a.pe = pair ? s->pe : nullptr;
    // energies are only written when asked for
    a.ce = trip && out ? (s->direct ? s->dir.ce : s->lo.ce) : nullptr;
    a.cc = trip && !s->direct ? s->lo.cc : nullptr;
    a.out = out;
    a.stride = stride;
    a.count_out = count_out;
    a.flags = s->flags;
    a.row = row;
    a.part = s->red_part;
    a.done = s->red_done;
    a.chunks = s->red_chunks;
    HIP_TRY(s, launch_reduce(s->st, a));
    return MTS_OK;
}

// Update kernel (see IntArgs).  xs_out: the drifted positions also go to the pair
// grid's sorted order (and are checked against the skin); null when a rebinning follows.
mts_status enqueue_int(mts_system *s, const double *f2prev, const double *f2cur, bool kick2,
                       bool kick3_end, bool kick3_start, bool drift, Pos4 *xs_out) {
    const double dt = s->p.dt, m = s->p.mass;
    IntArgs a{};
    a.n = s->n;
    a.x = s->xi;
    a.v = s->vi;
    a.f2prev = f2prev;
    a.f2cur = f2cur;
    a.f3 = s->f3;
    a.c2 = dt / (2.0 * m);
    a.c3 = (dt * (double)s->p.k) / (2.0 * m);
    a.dt = dt;
    a.cx = (dt * dt) / (2.0 * m);
    a.kick2 = kick2;
    a.kick3_end = kick3_end;
    a.kick3_start = kick3_start;
    a.drift = drift;
    a.open = s->direct ? 1 : 0;
    a.sd = s->direct ? s->dir.sd : s->lo.gt.sd;
    a.sys_of = s->sys_of;
    if (drift && xs_out) {
        a.inv_perm = s->lo.gp.inv_perm;
        a.xs = xs_out;
        a.x_ref = s->x_ref;
        a.half_skin2 = 0.25 * s->lo.skin * s->lo.skin;
    }
    a.flags = s->flags;
    HIP_TRY(s, launch_int(s->st, a));
    return MTS_OK;
}

// The list-build workgroups of a shared launch reserve the first tile class's LDS; past
// 64 KB (fewer than two triplet workgroups per CU) they run apart instead.
bool shared_launch(const mts_system *s) {
    return s->lo.skin > 0.0 && triplet_lds_bytes(s->lo.cls_cap[0], s->lo.list_cap, s->fp32) <= 64 * 1024;
}

// Rebins both grids at the internal positions, rebuilds the pair list and computes the
// triplet partial slots for mode (list mode); the caller's list force kernel then gathers F3.
mts_status enqueue_full_step_list(mts_system *s, bool energy, F3Mode mode) {
    MTS_TRY(enqueue_bin(s, kBinPair | kBinTriplet, s->xi, true));
    if (shared_launch(s)) {
        MTS_TRY(enqueue_triplet_and_list(s, energy, mode));
    } else {
        MTS_TRY(enqueue_list_build(s));
        MTS_TRY(enqueue_triplet(s, nullptr, nullptr, 0, energy, mode));
    }
    return MTS_OK;
}

// Forces at the internal positions x^0 of a call: F3 into s->f3, F2 into f2.
mts_status enqueue_entry_forces(mts_system *s, double *f2, bool energy) {
    if (s->direct) {
        MTS_TRY(enqueue_direct_pair(s, s->xi, f2, energy));
        MTS_TRY(enqueue_direct_triplet(s, s->xi, s->f3, energy));
    } else if (s->lo.skin > 0.0) {
        const F3Mode mode = cycle_mode(s, true);
        MTS_TRY(enqueue_full_step_list(s, energy, mode));
        Fused g;
        if (s->lo.cfg.gather_apart)
            HIP_TRY(s, launch_triplet_gather(s->st, s->n, s->pf, s->lo.gt.perm, s->f3, s->flags));
        else
            g.gather3 = true;
        MTS_TRY(enqueue_pair_list(s, s->lo.gp.xs, f2, g, true));
    } else {
        MTS_TRY(enqueue_bin(s, kBinPair | kBinTriplet, s->xi, false));
        MTS_TRY(enqueue_pair(s, f2));
        MTS_TRY(enqueue_triplet(s, s->f3, nullptr, 0, energy, cycle_mode(s, true)));
    }
    return MTS_OK;
}

// One outer cycle of Algorithm 2 on the internal copies xi, vi.  On entry F2 of the
// cycle's first position x^0 is in f2[0] and F3(x^0) in s->f3; on exit F2(x^k) is in
// f2[k % 2] and F3(x^k) in s->f3, with the closing F3 half kick applied.
// With a pair list (launches per cycle: k + 6, plus 1 with energies; k + 5 for a cycle that
// continues a call when k >= 2):
//   step 0:          k_int: opening F3 kick, drift to x^1 (also into sorted buffer B) --
//                    for a cycle that continues a call (k >= 2), done by the previous
//                    cycle's closing launch instead
//   x^i, 0 < i < k:  k_pair_list at x^i: F2(x^i), then kick2 of step i-1 and the drift
//                    of step i, positions ping-ponging between sorted buffers A and B
//   x^k:             rebin both grids (4 launches; a first binning pass fused into the
//                    last k_pair_list measured slower: its atomics with return stall
//                    the force kernel's few waves); one launch for the triplet partial
//                    slots of x^k and the new pair list; k_pair_list at x^k: F2(x^k),
//                    F3(x^k) gathered from the slots, last kick2 and the closing F3 kick
//                    (and, k >= 2, the next cycle's opening kick and first drift)
// Without a list (skin 0) every step rebins the pair grid and runs the tile kernel.
// DirectSum: k_int and the all-pairs kernel every step, the all-triplets kernel and its
// gather at x^k.
// Nested r-RESPA (k_outer > 1): this is one mid cycle; full says whether x^k ends a full
// step (then the class-weighted pass over the whole cutoff set, whose slots hold
// F_in + k_outer F_out; otherwise the inner class alone); energies only at full steps.
mts_status enqueue_cycle(mts_system *s, double *f2_0, double *f2_1, bool energies, bool full,
                         bool cont) {
    const int k = s->p.k;
    const F3Mode mode = cycle_mode(s, full);
    if (!full) energies = false;
    double *f2[2] = {f2_0, f2_1};
    if (s->direct) {
        for (int i = 0; i < k; ++i) {
            double *prev = f2[(i + 1) & 1], *cur = f2[i & 1], *next = f2[(i + 1) & 1];
            MTS_TRY(enqueue_int(s, prev, cur, i > 0, false, i == 0, true, nullptr));
            MTS_TRY(enqueue_direct_pair(s, s->xi, next, energies && i == k - 1));
            if (i == k - 1) MTS_TRY(enqueue_direct_triplet(s, s->xi, s->f3, energies));
        }
        MTS_TRY(enqueue_int(s, f2[(k - 1) & 1], f2[k & 1], true, true, false, false, nullptr));
    } else if (s->lo.skin > 0.0) {
        Pos4 *buf[2] = {s->lo.gp.xs, s->lo.gp.xs2};  // x^i lives in buf[i & 1] for 0 < i < k
        // with k >= 2 the closing launch also opens the next cycle (its F3 half kick and
        // first drift, into the sorted-order v, F2(x^0) and buf[1]), so a cycle that
        // continues a call starts at step 1 without k_int
        const bool fuse = k >= 2;
        if (!(fuse && cont))
            MTS_TRY(enqueue_int(s, nullptr, f2[0], false, false, true, true, k > 1 ? buf[1] : nullptr));
        for (int i = 1; i < k; ++i) {
            // steps 2 .. k-2 keep v and F2 in the pair grid's sorted order (the order
            // holds until the rebinning at x^k): step 1 reads them in input order (in
            // sorted order after a fused opening), step k - 1 writes them (and x) back in
            // input order
            Fused u;
            u.kick2 = true;
            u.drift = true;
            u.in_sorted = i >= 2 || (fuse && cont);
            u.out_sorted = i <= k - 2;
            u.f2prev = u.in_sorted ? s->f2s[(i - 1) & 1] : f2[(i - 1) & 1];
            u.xs_out = i + 1 < k ? buf[(i + 1) & 1] : nullptr;  // x^k: a rebinning follows
            MTS_TRY(enqueue_pair_list(s, buf[i & 1], u.out_sorted ? s->f2s[i & 1] : f2[i & 1], u, false));
        }
        MTS_TRY(enqueue_full_step_list(s, energies, mode));
        Fused u;
        if (s->lo.cfg.gather_apart)
            HIP_TRY(s, launch_triplet_gather(s->st, s->n, s->pf, s->lo.gt.perm, s->f3, s->flags));
        else
            u.gather3 = true;
        u.kick2 = true;
        u.kick3_end = true;
        u.open_next = fuse;
        u.f2prev = f2[(k - 1) & 1];
        MTS_TRY(enqueue_pair_list(s, s->lo.gp.xs, f2[k & 1], u, energies));
    } else {
        for (int i = 0; i < k; ++i) {
            double *prev = f2[(i + 1) & 1], *cur = f2[i & 1], *next = f2[(i + 1) & 1];
            MTS_TRY(enqueue_int(s, prev, cur, i > 0, false, i == 0, true, nullptr));
            if (i == k - 1) {
                MTS_TRY(enqueue_bin(s, kBinPair | kBinTriplet, s->xi, false));
                MTS_TRY(enqueue_pair(s, next));
                MTS_TRY(enqueue_triplet(s, s->f3, nullptr, 0, energies, mode));
            } else {
                MTS_TRY(enqueue_bin(s, kBinPair, s->xi, false));
                MTS_TRY(enqueue_pair(s, next));
            }
        }
        MTS_TRY(enqueue_int(s, f2[(k - 1) & 1], f2[k & 1], true, true, false, false, nullptr));
    }
    if (energies) {
        MTS_TRY(enqueue_reduce(s, s->vi, true, true, s->e_buf, kNE, s->row, nullptr));
    }
    return MTS_OK;
}

// Captures one cycle into an executable graph (kernels only: no memset or copy nodes).
mts_status capture_cycle(mts_system *s, bool energies, int parity, bool full, bool cont) {
    double *fa = parity ? s->f2b : s->f2a, *fb = parity ? s->f2a : s->f2b;
    HIP_TRY(s, hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    mts_status r = enqueue_cycle(s, fa, fb, energies, full, cont);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->st, &g);
    if (r != MTS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(s, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->gexec[energies][parity][full][cont], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
    return MTS_OK;
}

mts_status respa_internal(mts_system *s, double *x, double *v, int64_t n_iter, double *e_full) {
    const int k = s->p.k;
    const int64_t cycles = n_iter / k;                     // mid cycles of k steps
    const int64_t full_steps = n_iter / ((int64_t)k * s->k2);
    const bool energies = e_full != nullptr;
    const int64_t bytes = 3 * s->n * (int64_t)sizeof(double);
    if (energies && s->e_rows < full_steps + 1) {
        // grow the energy record buffer; graphs holding the old pointer are dropped
        drop_graphs(s);
        if (s->e_buf) HIP_TRY(s, hipFree(s->e_buf));
        s->e_buf = nullptr;
        s->e_rows = 0;
        HIP_TRY(s, dalloc(&s->e_buf, (size_t)(full_steps + 1) * s->nsys * kNE));
        s->e_rows = full_steps + 1;
    }
    if (bytes > 0) {
        HIP_TRY(s, hipMemcpyAsync(s->xi, x, bytes, hipMemcpyDeviceToDevice, s->st));
        HIP_TRY(s, hipMemcpyAsync(s->vi, v, bytes, hipMemcpyDeviceToDevice, s->st));
    }
    // Algorithm 2, lines 1-2: F2(x^0), F3(x^0); energies of x^0 in row 0
    MTS_TRY(enqueue_entry_forces(s, s->f2a, energies));
    if (energies) {
        HIP_TRY(s, launch_set_int(s->st, s->row, 0));
        MTS_TRY(enqueue_reduce(s, s->vi, true, true, s->e_buf, kNE, s->row, nullptr));
    }
    const bool graph = s->use_graph && !s->timing;
    for (int64_t c = 0; c < cycles; ++c) {
        const int parity = (k & 1) ? (int)(c & 1) : 0;
        const bool full = (c + 1) % s->k2 == 0;
        const bool e = energies && full;
        const bool cont = c > 0;  // the previous cycle of this call opened this one
        if (graph) {
            if (!s->gexec[e][parity][full][cont]) MTS_TRY(capture_cycle(s, e, parity, full, cont));
            HIP_TRY(s, hipGraphLaunch(s->gexec[e][parity][full][cont], s->st));
        } else {
            MTS_TRY(enqueue_cycle(s, parity ? s->f2b : s->f2a, parity ? s->f2a : s->f2b, e, full, cont));
        }
    }
    if (bytes > 0) {
        HIP_TRY(s, hipMemcpyAsync(x, s->xi, bytes, hipMemcpyDeviceToDevice, s->st));
        HIP_TRY(s, hipMemcpyAsync(v, s->vi, bytes, hipMemcpyDeviceToDevice, s->st));
    }
    if (energies)
        HIP_TRY(s, hipMemcpyAsync(e_full, s->e_buf, sizeof(double) * (size_t)(full_steps + 1) * s->nsys * kNE,
                                  hipMemcpyDeviceToDevice, s->st));
    return MTS_OK;
}

double lj_energy(double r2, double eps, double sigma) {
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

// ---- autotuning (see mts_autotune)

std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}

// Tuned configurations of this process, keyed by the shape of the problem.
std::map<std::string, std::pair<Config, double>> &tune_cache() {
    static std::map<std::string, std::pair<Config, double>> c;
    return c;
}

std::string shape_key(const mts_system *s) {
    std::string k;
    char buf[160];
    snprintf(buf, sizeof buf, "%.17g|%.17g|%.17g|%.17g|%.17g|%.17g|%.17g|%d|%d|%d|%d|%.17g",
             s->p.epsilon, s->p.sigma, s->p.rc_pair, s->p.nu, s->p.rc_triplet, s->p.mass, s->p.dt,
             s->p.k, s->p.precision, s->nsys, s->k2, s->p.rc_triplet_inner);
    k = buf;
    for (const SysDesc &d : s->base) {
        snprintf(buf, sizeof buf, "|%lld:%.17g,%.17g,%.17g", (long long)d.n, d.L[0], d.L[1], d.L[2]);
        k += buf;
    }
    return k;
}

// Largest triplet tile, forward-neighbour candidate list, pair tile and pair-list row
// seen on positions x with the current layout (the kernels record them with atomic
// maxima; a capacity overflow raised meanwhile is cleared, the maxima are what counts).
mts_status observe(mts_system *s, const double *x, int obs[4], std::vector<int> &tile) {
    HIP_TRY(s, hipMemsetAsync(s->stats, 0, 4 * sizeof(int), s->st));
    HIP_TRY(s, hipMemsetAsync(s->tile_obs, 0, sizeof(int) * s->nsys, s->st));
    s->collect_stats = true;
    mts_status r = enqueue_bin(s, kBinPair | kBinTriplet, x, false);
    if (r == MTS_OK) r = enqueue_list_build(s);
    if (r == MTS_OK) r = enqueue_triplet(s, nullptr, nullptr, 0, false);
    s->collect_stats = false;
    MTS_TRY(r);
    HIP_TRY(s, hipMemcpyAsync(obs, s->stats, 4 * sizeof(int), hipMemcpyDeviceToHost, s->st));
    tile.assign(s->nsys, 0);
    HIP_TRY(s, hipMemcpyAsync(tile.data(), s->tile_obs, sizeof(int) * s->nsys, hipMemcpyDeviceToHost, s->st));
    HIP_TRY(s, hipStreamSynchronize(s->st));
    HIP_TRY(s, hipMemset(s->flags, 0, sizeof(int)));
    HIP_TRY(s, hipMemset(s->tile_obs, 0, sizeof(int) * s->nsys));
    return MTS_OK;
}

// Capacities for the observed maxima, with room for the fluctuations of a run.
void caps_from_observed(Config &c, const int obs[4], const std::vector<int> &tile) {
    // margins against growth during the run: generous by default; thin with c.tight
    // (a tuning choice: smaller tiles and lists can buy a workgroup per CU, and an overflow
    // is reported and enlarged like any other)
    const double ft = c.tight ? 1.04 : 1.15, fl = c.tight ? 1.05 : 1.2;
    const int at = c.tight ? 8 : 16, al = c.tight ? 4 : 8;
    c.tile_need.resize(tile.size());
    for (size_t q = 0; q < tile.size(); ++q) c.tile_need[q] = (int)std::ceil(ft * tile[q]) + at;
    c.list_cap = std::min(kMaxListCap, round_up((int)std::ceil(fl * obs[1]) + al, 16));
    c.pair_cap = std::min(2048, round_up((int)std::ceil(1.15 * obs[2]) + 16, 32));
    if (c.skin > 0.0) c.nl_cap = std::min(2048, round_up((int)std::ceil(1.2 * obs[3]) + 16, 32));
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
    const double rc_max = std::max(params->rc_pair, params->rc_triplet);
    std::vector<SysDesc> base;
    int64_t p0 = 0;
    double lmin = INFINITY;
    for (int q = 0; q < n_systems; ++q) {
        SysDesc d{};
        if (n_particles[q] < 0) return MTS_ERR_INVALID_ARG;
        for (int k = 0; k < 3; ++k) {
            const double L = box[3 * q + k];
            if (!finite_pos(L)) return MTS_ERR_INVALID_ARG;
            if (params->method == MTS_CUTOFF && !(L > 2.0 * rc_max * kCellMargin))
                return MTS_ERR_BOX_TOO_SMALL;
            d.L[k] = L;
            d.iL[k] = 1.0 / L;
            lmin = std::min(lmin, L);
        }
        d.p0 = p0;
        d.n = n_particles[q];
        p0 += d.n;
        base.push_back(d);
    }
    if (p0 >= (int64_t)1 << 30) return MTS_ERR_UNSUPPORTED;

    mts_system *s = new mts_system();
    s->p = *params;
    s->direct = params->method == MTS_DIRECT;
    s->k2 = std::max(1, (int)params->k_outer);
    s->nsys = n_systems;
    s->n = p0;
    s->st = (hipStream_t)stream;
    s->fp32 = params->precision == MTS_FP32;
    s->base = base;
    s->lmin = lmin;
    s->ushift = params->lj_energy_shift
                    ? lj_energy(params->rc_pair * params->rc_pair, params->epsilon, params->sigma)
                    : 0.0;
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            s->max_lds = (size_t)lds;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            lds > 0)
            s->lds_per_cu = (size_t)lds;
        else
            s->lds_per_cu = s->max_lds;
        // keep room for the kernels' static LDS
        s->max_lds = s->max_lds > kStaticLdsReserve ? s->max_lds - kStaticLdsReserve : s->max_lds;
        if (configure_kernel_lds(s->max_lds) != hipSuccess) s->max_lds = 64 * 1024 - kStaticLdsReserve;
        (void)hipGetLastError();  // do not leave a failed attribute call as a sticky error
    }
    // Default configuration.  Pair-list skin: the requested one, by default
    // max(0.3 sigma, 12 k dt sqrt(eps/m)) (room for particles at four times a typical
    // thermal speed of LJ fluids); triplet cells of edge >= rc3; 16 lanes per particle.
    Config cfg;
    // F3 gathered apart for large systems: the scattered reads of the fused gather cost
    // more than a launch there (1M particles: +2.3 % MD steps/s; 32,000: -1.4 %)
    cfg.gather_apart = s->n >= (int64_t)1 << 17;
    cfg.skin = effective_skin(
        s, params->skin > 0.0
               ? params->skin
               : std::max(0.3 * params->sigma,
                          12.0 * params->k * params->dt * std::sqrt(params->epsilon / params->mass)));
    mts_status a = alloc_all(s);
    if (a == MTS_OK) a = s->direct ? setup_direct(s) : build_layout(s, cfg, s->lo);
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
    if (sys->direct) return fail(sys, MTS_ERR_UNSUPPORTED, "DirectSum handles keep no cells");
    if (!x && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x is NULL");
    return enqueue_bin(sys, kBinPair | kBinTriplet, x, false);
}

mts_status mts_compute_pair_forces(mts_system *sys, const double *x, double *f2, double *ew) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !f2) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or f2 is NULL");
    if (sys->direct) {
        MTS_TRY(enqueue_direct_pair(sys, x, f2, ew != nullptr));
    } else {
        MTS_TRY(enqueue_bin(sys, kBinPair, x, false));
        MTS_TRY(enqueue_pair(sys, f2));
    }
    if (ew) MTS_TRY(enqueue_reduce(sys, nullptr, true, false, ew, 2, nullptr, nullptr));
    return MTS_OK;
}

mts_status mts_compute_triplet_forces(mts_system *sys, const double *x, double *f3, double *ew) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !f3) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or f3 is NULL");
    if (sys->direct) {
        MTS_TRY(enqueue_direct_triplet(sys, x, f3, ew != nullptr));
    } else {
        MTS_TRY(enqueue_bin(sys, kBinTriplet, x, false));
        MTS_TRY(enqueue_triplet(sys, f3, nullptr, 0, ew != nullptr));
    }
    if (ew) MTS_TRY(enqueue_reduce(sys, nullptr, false, true, ew, 2, nullptr, nullptr));
    return MTS_OK;
}

mts_status mts_respa_step(mts_system *sys, double *x, double *v, int64_t n_iter, double *e_full) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !v) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or v is NULL");
    if (n_iter < 0) return fail(sys, MTS_ERR_INVALID_ARG, "n_iter < 0");
    if (n_iter % ((int64_t)sys->p.k * sys->k2) != 0)
        return fail(sys, MTS_ERR_NOT_MULTIPLE_OF_K,
                    "n_iter must be a multiple of k (Sec. 4.1), times k_outer when nested");
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
        case MTS_OPT_LIST_LANES:
            if (value != 4 && value != 8 && value != 16)
                return fail(sys, MTS_ERR_INVALID_ARG, "list lanes must be 4, 8 or 16");
            HIP_TRY(sys, hipStreamSynchronize(sys->ist));
            HIP_TRY(sys, hipStreamSynchronize(sys->st));
            drop_graphs(sys);  // captured list launches carry the old lane count
            sys->lo.cfg.lanes = (int)value;
            return MTS_OK;
        case MTS_OPT_TILE_CLASSES: {
            if (value != 0 && value != 1)
                return fail(sys, MTS_ERR_INVALID_ARG, "tile classes option must be 0 or 1");
            if (sys->direct) return MTS_OK;  // no triplet tiles
            Config c = sys->lo.cfg;
            c.split = value != 0;
            return set_layout(sys, c);
        }
        case MTS_OPT_F3_GATHER_APART:
            if (value != 0 && value != 1)
                return fail(sys, MTS_ERR_INVALID_ARG, "F3 gather option must be 0 or 1");
            HIP_TRY(sys, hipStreamSynchronize(sys->st));
            drop_graphs(sys);  // captured cycles carry the old placement
            sys->lo.cfg.gather_apart = value != 0;
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
    if (flags & (kFlagStageOverflow | kFlagListOverflow | kFlagPairList)) {
        Layout &lo = sys->lo;
        const int old_s = lo.stage_cap, old_l = lo.list_cap, old_p = lo.pair_cap, old_n = lo.nl_cap;
        const std::vector<int> old_need = lo.cfg.tile_need;
        bool triplet_tile = false;  // a triplet tile overflowed (else a pair tile did)
        if (flags & kFlagStageOverflow) {
            // triplet tiles: every overflowing system recorded its size; pair tiles double
            std::vector<int> obs(sys->nsys, 0);
            HIP_TRY(sys, hipMemcpy(obs.data(), sys->tile_obs, sizeof(int) * sys->nsys, hipMemcpyDeviceToHost));
            HIP_TRY(sys, hipMemset(sys->tile_obs, 0, sizeof(int) * sys->nsys));
            for (int q = 0; q < sys->nsys; ++q)
                if (obs[q] > 0) {
                    lo.cfg.tile_need[q] = std::max(lo.cfg.tile_need[q], (int)std::ceil(1.15 * obs[q]) + 16);
                    triplet_tile = true;
                }
            lo.pair_cap = std::min(4096, 2 * lo.pair_cap);
        }
        // what cannot grow any further: forward lists at their 256-entry limit (list
        // positions are packed in 8 bits), or a tile and lists beyond a workgroup's LDS
        bool stuck = (flags & kFlagListOverflow) && old_l >= kMaxListCap;
        if (flags & kFlagListOverflow) lo.list_cap = std::min(kMaxListCap, 2 * lo.list_cap);
        if (classify(sys, lo) != MTS_OK) {  // beyond the LDS of a workgroup: keep the old sizes
            lo.cfg.tile_need = old_need;
            lo.list_cap = old_l;
            (void)classify(sys, lo);
            stuck = true;
        }
        MTS_TRY(upload_classes(sys, lo));
        // a pair tile as large as a workgroup's LDS allows where doubling does not fit; an
        // overflowing pair tile that cannot grow is as stuck as a full list
        if (pair_lds_bytes(lo.pair_cap) > sys->max_lds)
            lo.pair_cap = std::max(old_p, (int)(sys->max_lds / pair_lds_bytes(1)) / 32 * 32);
        if ((flags & kFlagStageOverflow) && !triplet_tile && lo.pair_cap == old_p) stuck = true;
        if (flags & kFlagPairList) {
            const int cap = std::min(4096, 2 * sys->lo.nl_cap);
            int *nb = nullptr;
            if (dalloc(&nb, (size_t)sys->n * cap) == hipSuccess) {
                (void)hipFree(sys->lo.nbr);
                sys->lo.nbr = nb;
                sys->lo.nl_cap = cap;
            }
        }
        sys->lo.cfg.list_cap = sys->lo.list_cap;
        sys->lo.cfg.pair_cap = sys->lo.pair_cap;
        sys->lo.cfg.nl_cap = sys->lo.nl_cap;
        drop_graphs(sys);  // captured launches carry the old sizes and pointers
        char buf[400];
        snprintf(buf, sizeof buf,
                 "capacity overflow (flags %d): triplet tile %d -> %d, pair tile %d -> %d, "
                 "neighbour list %d -> %d, pair list %d -> %d; results since the last sync "
                 "are invalid%s",
                 flags, old_s, sys->lo.stage_cap, old_p, sys->lo.pair_cap, old_l, sys->lo.list_cap, old_n,
                 sys->lo.nl_cap,
                 stuck ? "; a tile or the forward lists cannot grow further (lists are "
                         "limited to 256 entries, tiles and lists to a workgroup's LDS)"
                       : "");
        return fail(sys, stuck ? MTS_ERR_UNSUPPORTED : MTS_ERR_CAPACITY, buf);
    }
    if (flags & kFlagSkin) {
        // the next call runs with a doubled skin (as far as the boxes allow)
        const double old_skin = sys->lo.skin;
        Config c = sys->lo.cfg;
        c.skin = effective_skin(sys, 2.0 * old_skin);
        if (c.skin > old_skin) {
            // the pair grid's cells and the list radius grow with the skin: pair tiles and
            // list rows observed on the old grid (autotuned capacities) may no longer fit,
            // so both are sized again for the new one
            c.pair_cap = 0;
            c.nl_cap = 0;
            (void)set_layout(sys, c);
        }
        char buf[240];
        snprintf(buf, sizeof buf,
                 "a particle moved more than half the pair-list skin (%.3g) between full steps; "
                 "pair forces since the last sync may miss pairs; skin now %.3g", old_skin,
                 sys->lo.skin);
        return fail(sys, MTS_ERR_CAPACITY, buf);
    }
    if (flags & kFlagNonFinite) return fail(sys, MTS_ERR_NONFINITE, "non-finite force or energy");
    return MTS_OK;
}

const char *mts_last_error(const mts_system *sys) { return sys ? sys->err.c_str() : ""; }

mts_status mts_get_grid(const mts_system *sys, int32_t system, int32_t n_cells[3]) {
    if (!sys || !n_cells || system < 0 || system >= sys->nsys) return MTS_ERR_INVALID_ARG;
    if (sys->direct) return MTS_ERR_UNSUPPORTED;
    for (int k = 0; k < 3; ++k) n_cells[k] = sys->lo.gt.hsd[system].nc[k];
    return MTS_OK;
}

mts_status mts_get_cell_index(mts_system *sys, int32_t *cell) {
    if (!sys || (!cell && sys->n > 0)) return MTS_ERR_INVALID_ARG;
    if (sys->direct) return fail(sys, MTS_ERR_UNSUPPORTED, "DirectSum handles keep no cells");
    HIP_TRY(sys, launch_local_cell_index(sys->st, sys->n, sys->lo.gt.cell_of, sys->lo.gt.sd, sys->sys_of, cell));
    return MTS_OK;
}

mts_status mts_count_triplets(mts_system *sys, const double *x, int64_t *count) {
    if (!sys || !count || (!x && sys->n > 0)) return MTS_ERR_INVALID_ARG;
    if (sys->direct) {  // every triplet of each system: C(n, 3)
        int64_t t = 0;
        for (const SysDesc &d : sys->base) t += d.n * (d.n - 1) * (d.n - 2) / 6;
        *count = t;
        return MTS_OK;
    }
    MTS_TRY(enqueue_bin(sys, kBinTriplet, x, false));
    MTS_TRY(enqueue_triplet(sys, nullptr, nullptr, 0, false));
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
    if (sys->direct) return fail(sys, MTS_ERR_UNSUPPORTED, "DirectSum: every i < j < k is a triplet");
    HIP_TRY(sys, hipMemsetAsync(sys->list_n, 0, sizeof(unsigned long long), sys->st));
    MTS_TRY(enqueue_bin(sys, kBinTriplet, x, false));
    MTS_TRY(enqueue_triplet(sys, nullptr, ijk, cap, false));
    unsigned long long total = 0;
    HIP_TRY(sys, hipMemcpyAsync(&total, sys->list_n, sizeof(unsigned long long), hipMemcpyDeviceToHost, sys->st));
    MTS_TRY(mts_sync(sys));
    *n = (int64_t)total;
    return MTS_OK;
}

static mts_status time_cycles(mts_system *s, const double *x, const double *v, double *tx,
                              double *tv, int cycles, double &ms) {
    const int64_t k = (int64_t)s->p.k * s->k2;  // one full step
    const int64_t bytes = 3 * s->n * (int64_t)sizeof(double);
    HIP_TRY(s, hipMemcpyAsync(tx, x, bytes, hipMemcpyDeviceToDevice, s->st));
    HIP_TRY(s, hipMemcpyAsync(tv, v, bytes, hipMemcpyDeviceToDevice, s->st));
    MTS_TRY(mts_respa_step(s, tx, tv, k, nullptr));  // warm-up: captures the cycle graphs
    MTS_TRY(mts_sync(s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(s, hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(s, he, "hipEventCreate");
    }
    mts_status r = MTS_OK;
    if (hipEventRecord(e0, s->st) != hipSuccess) r = fail(s, MTS_ERR_HIP, "hipEventRecord");
    if (r == MTS_OK) r = mts_respa_step(s, tx, tv, (int64_t)cycles * k, nullptr);
    if (r == MTS_OK && hipEventRecord(e1, s->st) != hipSuccess) r = fail(s, MTS_ERR_HIP, "hipEventRecord");
    if (r == MTS_OK) r = mts_sync(s);
    float t = 0.0f;
    if (r == MTS_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) r = fail(s, MTS_ERR_HIP, "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ms = (double)t / cycles;
    return r;
}

static void fill_tuning(const mts_system *s, mts_tuning *out) {
    const Config &c = s->lo.cfg;
    out->skin = c.skin;
    out->cell_factor = c.cell_factor;
    out->list_lanes = c.lanes;
    out->stage_cap = s->lo.stage_cap;
    out->list_cap = s->lo.list_cap;
    out->pair_cap = s->lo.pair_cap;
    out->nl_cap = s->lo.nl_cap;
    out->cycle_ms = s->tuned_ms;
    out->trials = s->tuned_trials;
    out->shared_launch = shared_launch(s) ? 1 : 0;
    out->tile_classes = s->lo.ncls;
    out->tight_caps = c.tight ? 1 : 0;
    out->f3_gather_apart = c.gather_apart ? 1 : 0;
    out->triplet_workgroups_per_cu = s->direct || s->lo.ncls == 0 ? 0 : s->lo.cls_occ[0];
}

mts_status mts_get_tuning(const mts_system *sys, mts_tuning *out) {
    if (!sys || !out) return MTS_ERR_INVALID_ARG;
    fill_tuning(sys, out);
    return MTS_OK;
}

mts_status mts_autotune(mts_system *sys, const double *x, const double *v, int32_t budget_ms,
                        mts_tuning *out) {
    if (!sys) return MTS_ERR_INVALID_ARG;
    if ((!x || !v) && sys->n > 0) return fail(sys, MTS_ERR_INVALID_ARG, "x or v is NULL");
    if (sys->timing) return fail(sys, MTS_ERR_INVALID_ARG, "kernel timing is enabled");
    MTS_TRY(mts_sync(sys));
    if (sys->direct) {  // nothing to choose: no cells, lists or capacities
        if (out) fill_tuning(sys, out);
        return MTS_OK;
    }
    const std::string key = shape_key(sys);
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            MTS_TRY(set_layout(sys, it->second.first));
            sys->tuned_ms = it->second.second;
            sys->tuned_trials = 0;
            if (out) fill_tuning(sys, out);
            return MTS_OK;
        }
    }
    if (sys->n == 0) {
        if (out) fill_tuning(sys, out);
        return MTS_OK;
    }
    const auto t_start = std::chrono::steady_clock::now();
    const double budget = budget_ms > 0 ? (double)budget_ms : 2000.0;
    double *tx = nullptr, *tv = nullptr;
    HIP_TRY(sys, dalloc(&tx, 3 * sys->n));
    if (dalloc(&tv, 3 * sys->n) != hipSuccess) {
        (void)hipFree(tx);
        return fail(sys, MTS_ERR_OOM, "autotune scratch");
    }
    // Smallest skin worth trying: a particle 1.5x faster than the fastest one of the input
    // must stay within half the skin over a whole outer cycle.
    double vmax = 0.0;
    {
        std::vector<double> hv(3 * sys->n);
        if (hipMemcpy(hv.data(), v, hv.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipFree(tx);
            (void)hipFree(tv);
            return fail(sys, MTS_ERR_HIP, "autotune: reading v");
        }
        for (int64_t i = 0; i < sys->n; ++i) {
            const double a = hv[3 * i], b = hv[3 * i + 1], c = hv[3 * i + 2];
            vmax = std::max(vmax, std::sqrt((a * a + b * b) + c * c));
        }
    }
    const double min_skin = 2.0 * 1.5 * vmax * sys->p.k * sys->p.dt;
    const Config start = sys->lo.cfg;
    int trials = 0;
    // One configuration: layout with heuristic capacities, capacities from the maxima
    // observed on x, then the timed cycles.  Returns the ms per cycle, or +inf when the
    // configuration does not fit (box, LDS) or overflowed during the run.
    auto trial = [&](Config c) -> std::pair<double, Config> {
        c.tile_need.clear();
        c.list_cap = c.pair_cap = c.nl_cap = 0;
        if (set_layout(sys, c) != MTS_OK) return {INFINITY, c};
        int obs[4] = {0, 0, 0, 0};
        std::vector<int> tile;
        if (observe(sys, x, obs, tile) != MTS_OK) return {INFINITY, c};
        caps_from_observed(c, obs, tile);
        if (set_layout(sys, c) != MTS_OK) return {INFINITY, c};
        ++trials;
        // enough cycles for about 4 ms of work (at least 3), timed twice: the faster run
        double ms = INFINITY, once = 0.0;
        int cycles = 3;
        for (int rep = 0; rep < 2; ++rep) {
            if (time_cycles(sys, x, v, tx, tv, cycles, once) != MTS_OK) {
                (void)mts_sync(sys);  // clears the flags and the error of an overflowed run
                return {INFINITY, sys->lo.cfg};
            }
            ms = std::min(ms, once);
            if (rep == 0 && once > 0.0) cycles = std::max(3, std::min(200, (int)std::ceil(4.0 / once)));
        }
        return {ms, sys->lo.cfg};
    };
    auto over_budget = [&]() {
        const double el = std::chrono::duration<double, std::milli>(
                              std::chrono::steady_clock::now() - t_start).count();
        return el > budget;
    };
    std::pair<double, Config> best = trial(start);
    // coordinate descent over the capacity margins, the pair-list skin, the triplet cell
    // size, the lanes per particle of the list force kernel and, for batches, the triplet
    // launch grouping (the knobs that moved the cycle most come first, so that a short
    // budget still reaches them)
    // capacities with thin margins (more triplet workgroups per CU where they then fit)
    if (!over_budget()) {
        Config c = best.second;
        c.tight = !c.tight;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    const double sg = sys->p.sigma;
    for (double sk : {0.15 * sg, 0.1 * sg, 0.2 * sg, 0.3 * sg, 0.5 * sg, 0.0}) {
        if (over_budget()) break;
        Config c = best.second;
        c.skin = effective_skin(sys, sk);
        if (c.skin == best.second.skin || (c.skin > 0.0 && c.skin < min_skin)) continue;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    for (double f : {1.0, 1.12, 1.25}) {
        if (over_budget()) break;
        Config c = best.second;
        if (c.cell_factor == f) continue;
        c.cell_factor = f;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    for (int g : {16, 8, 4}) {
        if (over_budget() || best.second.skin == 0.0) break;
        Config c = best.second;
        if (c.lanes == g) continue;
        c.lanes = g;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    // F3 gathered by its own kernel or inside the list force kernel
    if (!over_budget()) {
        Config c = best.second;
        c.gather_apart = !c.gather_apart;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    // batches: one triplet launch at the occupancy of the largest tile, or one launch per
    // tile class
    if (sys->nsys > 1 && !over_budget()) {
        Config c = best.second;
        c.split = !c.split;
        auto r = trial(c);
        if (r.first < 0.98 * best.first) best = r;
    }
    (void)hipFree(tx);
    (void)hipFree(tv);
    if (!std::isfinite(best.first)) {
        // nothing could be timed: back to the configuration the handle had
        MTS_TRY(set_layout(sys, start));
        return fail(sys, MTS_ERR_CAPACITY, "autotune: no configuration ran without overflow");
    }
    MTS_TRY(set_layout(sys, best.second));
    sys->tuned_ms = best.first;
    sys->tuned_trials = trials;
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_cache()[key] = {best.second, best.first};
    }
    if (out) fill_tuning(sys, out);
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
