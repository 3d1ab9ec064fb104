/*
 * mts.h -- C ABI of the MI355X (gfx950) library for two- plus three-body molecular
 * dynamics with r-RESPA multiple time stepping.
 *
 * The method (Martin et al., "The Multiple Time-Stepping Method for 3-Body
 * Interactions in High Performance Molecular Dynamics Simulations"):
 *   - pair force F2 = -grad of the Lennard-Jones 12-6 potential (Sec. 2.1), cut off
 *     at rc_pair, evaluated every step;
 *   - triplet force F3 = -grad of the Axilrod-Teller-Muto potential (Sec. 2.1) over
 *     every triplet whose three pairwise distances are all <= rc_triplet
 *     (Sec. 4.1 and 4.2.2), found through linked cells (Sec. 2.2, 4.1), evaluated
 *     once per outer step;
 *   - r-RESPA as the paper implements it (Sec. 4.1, Algorithm 2): F2 every step,
 *     F3 kicks of dt*s/(2m) every s-th step, s = k here.  Algorithm 1 (Sec. 2.3.1: full
 *     steps delta_t of P sub-steps each) is the same scheme with dt = delta_t / P, k = P;
 *   - optionally three time scales (mts_params.k_outer): the nested form of Sec. 2.3.1
 *     over two distance classes of triplets split at an intermediate cutoff (Sec. 5).
 *
 * Conventions shared by every call
 *   - Units: reduced Lennard-Jones units as in the paper's appendix table.
 *   - Positions, velocities and forces are FP64 device arrays [N][3], row-major
 *     (x, y, z of particle 0, then particle 1, ...), N = sum of n_particles[].
 *     Systems are concatenated in order.  Forces come back in this same order.
 *   - Boxes are orthorhombic and periodic.  Every edge must exceed twice the larger
 *     cutoff (so that each pair has at most one interacting image).
 *   - Cutoffs are inclusive: d^2 <= rc^2, with d the minimum-image displacement.
 *   - Pointers marked "dev" are device pointers (e.g. torch CUDA tensors on ROCm);
 *     "host" pointers are ordinary CPU memory.  The caller owns every pointer it
 *     passes and keeps it alive until the work is done; the library never frees
 *     caller memory.  The library owns cells, work buffers and force caches.
 *   - Asynchrony: calls validate on the host, enqueue work on the stream given at
 *     init and return without waiting, unless documented as synchronising.  Device
 *     side problems (capacity overflow, non-finite values) raise flags that the
 *     next mts_sync() reports.  A handle must not be used from two threads at once.
 *   - Return value: MTS_OK or a negative mts_status; mts_last_error() gives text.
 */
#ifndef MTS_H
#define MTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mts_system mts_system; /* opaque, library-owned */

typedef enum {
    MTS_OK = 0,
    MTS_ERR_INVALID_ARG = -1,       /* bad pointer, size or parameter */
    MTS_ERR_BOX_TOO_SMALL = -2,     /* a box edge is not above 2 * max(rc_pair, rc_triplet) */
    MTS_ERR_NOT_MULTIPLE_OF_K = -3, /* n_iter is not a multiple of k (Sec. 4.1) */
    MTS_ERR_CAPACITY = -4,          /* a cell neighbourhood or neighbour list overflowed */
    MTS_ERR_NONFINITE = -5,         /* a force or energy became NaN or infinite */
    MTS_ERR_HIP = -6,               /* a HIP runtime call failed */
    MTS_ERR_OOM = -7,               /* device allocation failed */
    MTS_ERR_UNSUPPORTED = -8        /* valid input this library does not handle */
} mts_status;

typedef enum {
    MTS_FP64 = 0, /* all force arithmetic in FP64 */
    MTS_FP32 = 1  /* ATM arithmetic in FP32; LJ arithmetic, cutoff geometry, accumulation,
                     integration and energy reductions in FP64 */
} mts_precision;

/* How interactions are found. */
typedef enum {
    MTS_CUTOFF = 0, /* periodic boxes; pairs within rc_pair, triplets with all three edges
                       within rc_triplet, through linked cells (Sec. 4.1, cutoff) */
    MTS_DIRECT = 1  /* DirectSum (Sec. 3.1, 4.1): every pair and every triplet of a system,
                       no cutoff and open boundaries (no images, positions never wrapped);
                       the cutoffs, skin and box are not used */
} mts_method;

/* Interaction and integration parameters (Sec. 2.1; appendix table). */
typedef struct {
    double epsilon;          /* LJ well depth epsilon_LJ */
    double sigma;            /* LJ length sigma_LJ */
    double rc_pair;          /* pair cutoff */
    double nu;               /* ATM coefficient nu_ATM */
    double rc_triplet;       /* three-body cutoff: all three edges <= rc_triplet */
    double mass;             /* particle mass m (uniform) */
    double dt;               /* inner time step delta t */
    double skin;             /* Verlet pair-list skin added to rc_pair (0: the default,
                                max(0.3 sigma, 12 k dt sqrt(epsilon/mass))); shrunk to fit
                                the box, no list below 0.05 sigma */
    int32_t k;               /* r-RESPA step-size factor s >= 1 (Sec. 4.1) */
    int32_t precision;       /* mts_precision */
    int32_t lj_energy_shift; /* 1: report U2 shifted by -U(rc_pair) per pair (forces unchanged) */
    int32_t method;          /* mts_method */
    int32_t k_outer;         /* nested r-RESPA over two triplet distance classes (Sec. 2.3.1
                                nested loops, applied to the intermediate cutoffs of Sec. 5):
                                0 or 1: off (Algorithm 2 with s = k); > 1: the outer class
                                (longest edge > rc_triplet_inner) kicks every k * k_outer
                                steps, the inner class (all edges <= rc_triplet_inner) every
                                k steps; MTS_CUTOFF only */
    double rc_triplet_inner; /* class split r_a: 0 < r_a < rc_triplet when k_outer > 1, else 0 */
} mts_params;

/* Energy record per system: kinetic K, LJ energy U2, ATM energy U3, pair virial W2,
 * triplet virial W3 (W = sum over interactions of x . F, so that the pressure is
 * (2K + W2 + W3) / (3V)). */
enum { MTS_NE = 5 };

/* Creates a handle for n_systems independent systems (periodic boxes, or open ones with
 * MTS_DIRECT).
 *   params       host, read during the call.
 *   n_particles  host [n_systems], each >= 0.
 *   box          host [n_systems][3], edge lengths (> 0; unused with MTS_DIRECT).
 *   stream       hipStream_t to enqueue on (NULL = default stream).
 *   out          host, receives the handle; release it with mts_destroy_system.
 * Fails with MTS_ERR_BOX_TOO_SMALL, MTS_ERR_INVALID_ARG, MTS_ERR_OOM, or
 * MTS_ERR_UNSUPPORTED (k_outer > 1 with MTS_DIRECT, or 2^30 particles or more); on
 * failure *out is NULL. */
mts_status mts_init_system(const mts_params *params, int32_t n_systems, const int64_t *n_particles,
                           const double *box, void *stream, mts_system **out);

/* Waits for queued work, then frees every library-owned buffer.  NULL is ignored. */
void mts_destroy_system(mts_system *sys);

/* Assigns particles to linked cells (Sec. 2.2, 4.1): wraps positions into the box,
 * computes each cell index and sorts particles by cell with a stable counting sort
 * (equal cells keep ascending particle order).  x is dev [N][3]; it is read, not
 * modified.  The force calls below bin by themselves; this call exists for the cell
 * inspection exports.  MTS_DIRECT handles keep no cells: MTS_ERR_UNSUPPORTED. */
mts_status mts_build_cells(mts_system *sys, const double *x);

/* F2(x): Lennard-Jones forces (Sec. 2.1; Algorithm 2, "calculate F2b"); with MTS_DIRECT
 * over every pair of a system, unshifted.
 *   x   dev [N][3] positions (need not be wrapped).
 *   f2  dev [N][3] output, overwritten.
 *   ew  dev [n_systems][2] output {U2, W2}, or NULL. */
mts_status mts_compute_pair_forces(mts_system *sys, const double *x, double *f2, double *ew);

/* F3(x): Axilrod-Teller-Muto forces over every triplet with all three edges
 * <= rc_triplet (Sec. 2.1, 4.1; Algorithm 2, "calculate F3b"), or with MTS_DIRECT over
 * every triplet i < j < k of a system.  Newton's third law is applied across each
 * triplet: every triplet is evaluated once.
 *   x   dev [N][3] positions.
 *   f3  dev [N][3] output, overwritten.
 *   ew  dev [n_systems][2] output {U3, W3}, or NULL. */
mts_status mts_compute_triplet_forces(mts_system *sys, const double *x, double *f3, double *ew);

/* Runs n_iter inner steps of r-RESPA (Sec. 4.1, Algorithm 2) in place.  Each outer
 * cycle (k inner steps, one F3 evaluation, its half kicks and the energy record) is one
 * captured HIP graph replayed on a library stream that is ordered after, and before, the
 * handle's stream (see MTS_OPT_CYCLE_GRAPH); the caller's x and v are copied in and out.
 * With k_outer > 1 (nested, three time scales) a full step spans S = k * k_outer inner
 * steps: the outer triplet class is evaluated and kicked (dt S / 2m) at its ends, the
 * inner class every k steps (dt k / 2m); at a full step both kicks fall together.
 * Otherwise S = k.
 *   x       dev [N][3] positions x^0 in, x^n out (wrapped into the box after each drift).
 *   v       dev [N][3] velocities v^0 in, v^n out.
 *   n_iter  number of inner steps, a multiple of S (else MTS_ERR_NOT_MULTIPLE_OF_K).
 *   e_full  dev [n_iter/S + 1][n_systems][MTS_NE] energies at x^0 and after every full
 *           step (only full steps have synchronised velocities; U3 and W3 cover both
 *           classes), or NULL.
 * Both forces are recomputed at x^0 on entry, as Algorithm 2 does, so two calls of
 * n and m steps equal one call of n + m steps.  Between full steps the pair forces come
 * from a Verlet list of radius rc_pair + skin built at every full step (see
 * mts_params.skin and mts_autotune); a particle that moves more than half the skin from
 * its position at the build is reported by the next mts_sync as MTS_ERR_CAPACITY (the
 * forces since may miss pairs; the skin is enlarged for the next call, and the pair tile
 * and list-row capacities are sized again for the coarser pair grid). */
mts_status mts_respa_step(mts_system *sys, double *x, double *v, int64_t n_iter, double *e_full);

/* Waits for the stream and reports device flags raised since the last mts_sync:
 * MTS_ERR_CAPACITY (the affected forces are wrong; the tile or list capacities, or the
 * pair-list skin when a particle outran half of it, are enlarged for the next call),
 * MTS_ERR_UNSUPPORTED (an overflow that no enlargement can cure: a forward-neighbour list
 * beyond its 256-entry limit, a triplet tile and lists or a pair tile beyond a
 * workgroup's LDS; the input is too dense for this library -- repeating the call fails
 * the same way) or
 * MTS_ERR_NONFINITE.  Clears the flags. */
mts_status mts_sync(mts_system *sys);

/* Text of the last error on this handle ("" if none); valid until the next call. */
const char *mts_last_error(const mts_system *sys);

/* Name of a status code. */
const char *mts_status_string(int32_t status);

/* ---- inspection exports (used by the parity tests) ---- */

/* Cell grid of one system: n_cells[0..2] along x, y, z (host out).  MTS_DIRECT:
 * MTS_ERR_UNSUPPORTED (no cells). */
mts_status mts_get_grid(const mts_system *sys, int32_t system, int32_t n_cells[3]);

/* After mts_build_cells: per-particle linear cell index (c_z * n_y + c_y) * n_x + c_x
 * within its own system's grid.  cell is dev [N] int32, in input particle order.
 * MTS_DIRECT: MTS_ERR_UNSUPPORTED. */
mts_status mts_get_cell_index(mts_system *sys, int32_t *cell);

/* Number of interacting triplets at x, summed over systems (MTS_DIRECT: the sum of
 * C(N, 3), no device work).  Synchronising; count is a host pointer. */
mts_status mts_count_triplets(mts_system *sys, const double *x, int64_t *count);

/* Lists the interacting triplets at x as particle-index triples (i<j<k, global
 * indices), in no particular order.  ijk is dev [cap][3] int32; *n (host) receives
 * the total count, which may exceed cap (then only cap rows are written).
 * Synchronising.  MTS_DIRECT (every i < j < k): MTS_ERR_UNSUPPORTED unless cap is 0. */
mts_status mts_list_triplets(mts_system *sys, const double *x, int32_t *ijk, int64_t cap,
                             int64_t *n);

/* ---- options ---- */

enum {
    /* 1 (default): mts_respa_step replays each outer cycle from a captured HIP graph on
     * an internal stream; 0: launches every kernel one by one (same kernels, same order,
     * bitwise-identical results). */
    MTS_OPT_CYCLE_GRAPH = 1,
    /* Lanes per particle of the list force kernel: 4, 8 or 16 (else MTS_ERR_INVALID_ARG).
     * mts_autotune searches this knob and sets it; results differ between lane counts
     * only by the order of the per-particle sums.  Takes effect from the next call. */
    MTS_OPT_LIST_LANES = 2,
    /* Triplet launches of a batch: 0 (default) one launch over every system; 1 one launch
     * per tile class (systems grouped by the workgroups per CU their tiles allow).
     * mts_autotune tries both for batches.  Results are bitwise the same either way. */
    MTS_OPT_TILE_CLASSES = 3,
    /* Where F3 is summed from the triplet partial slots at each full step: 1 by a kernel of
     * its own, 0 inside the list force kernel (default: 1 for 128 Ki particles and more).
     * mts_autotune tries both.  Results are bitwise the same either way (the same slot
     * order). */
    MTS_OPT_F3_GATHER_APART = 4
};

/* Sets an option (see the MTS_OPT_ constants).  MTS_ERR_INVALID_ARG for unknown options. */
mts_status mts_set_option(mts_system *sys, int32_t option, int64_t value);

/* ---- autotuning ---- */

/* A handle's tunable configuration. */
typedef struct {
    double skin;          /* Verlet pair-list skin in use (0: no list; the pair grid is
                             rebinned every inner step) */
    double cell_factor;   /* triplet cells have edges >= cell_factor * rc_triplet (>= 1) */
    int32_t list_lanes;   /* lanes per particle of the list force kernel (4, 8 or 16) */
    int32_t stage_cap;    /* largest triplet tile capacity (particles staged per workgroup)
                             over the tile classes */
    int32_t list_cap;     /* forward-neighbour list capacity per anchor particle */
    int32_t pair_cap;     /* pair tile capacity */
    int32_t nl_cap;       /* pair-list row capacity */
    int32_t trials;       /* configurations the last mts_autotune timed (0: cached/untuned) */
    int32_t shared_launch;/* 1: the pair list is built in the triplet kernel's launch */
    int32_t tile_classes; /* triplet launches per force evaluation: 1 by default (every
                             system in one launch); mts_autotune may group the systems of a
                             batch by the workgroups per CU their tile size allows, one
                             launch per group, when that measures faster */
    double cycle_ms;      /* measured ms per full step (k inner steps, k * k_outer when
                             nested; 0: untuned) */
    int32_t tight_caps;   /* 1: capacities sized from the observed maxima with thin margins
                             (mts_autotune keeps it when the smaller tiles and lists let
                             more triplet workgroups share a CU and that measures faster) */
    int32_t triplet_workgroups_per_cu; /* triplet workgroups one CU holds in the (first)
                             triplet launch at the current capacities (0: DirectSum) */
    int32_t f3_gather_apart; /* 1: F3 is summed from the triplet partial slots by a kernel
                             of its own at each full step (coalesced reads; by default for
                             128 Ki particles and more); 0: inside the list force kernel */
    int32_t pad_;         /* keeps the struct a multiple of 8 bytes */
} mts_tuning;

/* (MTS_DIRECT handles have nothing to tune: the call returns their configuration.)
 * Chooses, by measurement on the caller's input, the configuration that runs one outer
 * r-RESPA cycle fastest -- the role AutoPas's run-time algorithm selection plays for the
 * paper's CPU code (Sec. 4.1, cutoff implementation).  Candidates: pair-list skin
 * (none, 0.15, 0.3, 0.5 sigma; only skins that a particle 1.5 times faster than the
 * fastest one in v would not outrun in one outer cycle), triplet cell factor (1, 1.12,
 * 1.25) and list-kernel
 * lanes (16, 8, 4), searched one knob at a time from the current configuration; each
 * candidate gets tile and list capacities sized from the maxima observed on x, a warm-up
 * cycle and the faster of two timed runs of about 4 ms (at least 3 cycles each), and
 * replaces the best so far only if at least 2% faster.  The search stops once budget_ms
 * of wall time is spent (<= 0: 2000 ms).  It runs on copies: x, v (dev [N][3]) are read,
 * not modified.  The winner stays on the handle and is cached for the process by problem
 * shape (parameters, particle counts, boxes): a later call on a handle of that shape
 * applies it without timing.  Every configuration yields the same triplet and pair sets
 * and forces within the oracle tolerances.  Synchronising; out (host) may be NULL.
 * MTS_ERR_CAPACITY if no candidate ran without overflow (the handle then keeps its
 * previous configuration). */
mts_status mts_autotune(mts_system *sys, const double *x, const double *v, int32_t budget_ms,
                        mts_tuning *out);

/* The handle's current configuration (host out). */
mts_status mts_get_tuning(const mts_system *sys, mts_tuning *out);

/* ---- profiling hook ---- */

/* Turns per-launch timing of the two force kernels on or off (synchronising).  While on,
 * every launch of the triplet-force kernel and of the pair-force kernel is bracketed by
 * HIP events recorded on the handle's stream. */
mts_status mts_enable_kernel_timing(mts_system *sys, int32_t enable);

/* Synchronising.  For kernel class 0 (the triplet-force launch, which also builds the
 * pair list when mts_tuning.shared_launch is 1) and 1 (pair forces): launches[c]
 * receives the number of timed launches since the last call and ms[c] their summed
 * duration in milliseconds (host arrays of 2).  Resets the counters. */
mts_status mts_kernel_times(mts_system *sys, int64_t launches[2], double ms[2]);

/* ---- without a handle, without allocating ---- */

/* Device memory this entry point works in: one static array per GPU (16 MiB). */
#define MTS_STATIC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: the triplet forces F3 (and, with ew,
 * {U3, W3}) of one periodic system, as mts_compute_triplet_forces computes them on a
 * one-system handle with the same params, but with no handle and no allocation.  The
 * cell grid, partial-force slots and counters live in a static device array of
 * MTS_STATIC_SCRATCH_BYTES that each GPU holds until the process ends (about 390 bytes
 * per particle plus 32 per cell: roughly 40,000 particles at liquid density).
 *   params  only epsilon/sigma/rc_pair (box check), nu, rc_triplet and precision are
 *           used; method must be MTS_CUTOFF and k_outer <= 1 (else MTS_ERR_UNSUPPORTED)
 *   n       particles (>= 0); box: host [3] edges, each > 2 max(rc_pair, rc_triplet)
 *   x       dev [n][3] FP64 positions, any image; f3: dev [n][3] out; ew: dev [2] out or NULL
 *   stream  HIP stream (NULL: the default stream) the work is enqueued on
 * Synchronising: waits for the stream and returns MTS_OK, MTS_ERR_CAPACITY (the system
 * needs more than MTS_STATIC_SCRATCH_BYTES, or a cell neighbourhood or forward list
 * outgrew the capacities sized from the mean density: f3 is then invalid),
 * MTS_ERR_NONFINITE, MTS_ERR_BOX_TOO_SMALL, MTS_ERR_INVALID_ARG or MTS_ERR_HIP.
 * Every call on one GPU works in that GPU's one array: calls that overlap on a GPU
 * (other threads, other streams) race and must be serialised by the caller. */
mts_status mts_compute_triplet_forces_static(const mts_params *params, int64_t n,
                                             const double box[3], const double *x,
                                             double *f3, double *ew, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MTS_H */
