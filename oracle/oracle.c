/*
 * oracle.c -- plain FP64 CPU reference for Lennard-Jones + Axilrod-Teller-Muto
 * molecular dynamics with the r-RESPA multiple time-stepping loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file: only the test suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or helper with the HIP library.
 *
 * Everything is a literal, slow, exhaustive definition:
 *   - pairs    P = { i<j : |d_ij|^2 <= rc_pair^2 }                     (Sec. 2.1, LJ)
 *   - triplets T = { i<j<k : all three squared distances <= rc3^2 }      (Sec. 4.2.2:
 *                  all three pairwise distances must lie within the cutoff)
 *   - F = -grad(Phi)                                                      (Sec. 2, Eq. 2)
 *   - r-RESPA as the paper implements it (Sec. 4.1, Algorithm 2)
 *   - textbook velocity Verlet (Stoermer-Verlet, Sec. 2.3) as an independent integrator.
 *
 * Periodic boundaries (the paper's Cutoff runs use them, Sec. 4.2).  Readings where
 * the paper is silent:
 *   - positions are wrapped into the box by  w = x - L*floor(x/L);
 *   - a pair displacement is the minimum image  d = (x_q - x_p) - L*rint((x_q - x_p)/L);
 *   - a squared distance is  ((dx*dx + dy*dy) + dz*dz)  in that order;
 *   - cutoffs are inclusive:  d^2 <= rc*rc;
 *   - a triplet needs its three minimum-image displacements to close the triangle,
 *     which always holds when every box edge exceeds 3*rc; boxes must exceed 2*rc;
 *   - the reported LJ energy may be shifted by -U(rc) per included pair; forces are
 *     plainly truncated.  ATM energy is not shifted.
 * Compile with -ffp-contract=off so that no expression is fused into an FMA.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID_ARG (-1)
#define ORC_ERR_BOX_TOO_SMALL (-2)
#define ORC_ERR_NOT_MULTIPLE_OF_K (-3)
#define ORC_ERR_NONFINITE (-5)
#define ORC_ERR_OOM (-7)

/* ------------------------------------------------------------------ geometry */

static double wrap1(double x, double L) { return x - L * floor(x / L); }

static double mic1(double d, double L) { return d - L * rint(d / L); }

/* Minimum-image displacement from particle p to particle q, and its squared length. */
static double disp2(const double *xp, const double *xq, const double *L, double d[3]) {
    for (int c = 0; c < 3; ++c) d[c] = mic1(xq[c] - xp[c], L[c]);
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

static double dot3(const double *a, const double *b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static int box_ok(const double *L, double rc) {
    for (int c = 0; c < 3; ++c)
        if (!(L[c] > 2.0 * rc)) return 0;
    return 1;
}

static double *wrapped_copy(int64_t n, const double *x, const double *L) {
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    if (!w) return NULL;
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) w[3 * i + c] = wrap1(x[3 * i + c], L[c]);
    return w;
}

int orc_wrap(int64_t n, const double *x, const double *L, double *out) {
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) out[3 * i + c] = wrap1(x[3 * i + c], L[c]);
    return ORC_OK;
}

/* Linked-cell index of every particle (Sec. 2.2 / 4.1: particles are assigned to
 * cells by position).  Cell coordinate c_d = min(n_d - 1, floor(w_d * (n_d / L_d)))
 * on the wrapped position w; linear index (c_z * n_y + c_y) * n_x + c_x. */
int orc_cell_index(int64_t n, const double *x, const double *L, const int32_t *nc, int32_t *cell) {
    double q[3];
    for (int c = 0; c < 3; ++c) {
        if (nc[c] < 1) return ORC_ERR_INVALID_ARG;
        q[c] = (double)nc[c] / L[c];
    }
    for (int64_t i = 0; i < n; ++i) {
        int cc[3];
        for (int c = 0; c < 3; ++c) {
            double w = wrap1(x[3 * i + c], L[c]);
            int v = (int)floor(w * q[c]);
            if (v > nc[c] - 1) v = nc[c] - 1;
            if (v < 0) v = 0;
            cc[c] = v;
        }
        cell[i] = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ potentials */

/* Lennard-Jones 12-6 (Sec. 2.1): phi2(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6].
 * Given d = x_j - x_i with r^2 = |d|^2, returns phi2 and sets *fr so that the force
 * on j is fr * d and the force on i is -fr * d:  fr = -(dphi2/dr) / r
 *   = 24 eps [2 (sigma/r)^12 - (sigma/r)^6] / r^2.  The pair virial d . F_j is fr * r^2. */
static double lj(double r2, double eps, double sigma, double *fr) {
    double s2 = (sigma * sigma) / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    *fr = 24.0 * eps * (2.0 * s12 - s6) / r2;
    return 4.0 * eps * (s12 - s6);
}

/* Axilrod-Teller-Muto (Sec. 2.1):
 *   phi3 = nu (1 + 3 cos(th_i) cos(th_j) cos(th_k)) / (r_ij r_ik r_jk)^3,
 * th_i the angle at i between the edges towards j and k, and so on.
 * u = x_j - x_i, w = x_k - x_i, v = x_k - x_j (minimum images closing the triangle). */
static double atm_energy(const double *u, const double *w, const double *v, double nu) {
    double rij = sqrt(dot3(u, u)), rik = sqrt(dot3(w, w)), rjk = sqrt(dot3(v, v));
    double mu[3] = {-u[0], -u[1], -u[2]};
    double cos_i = dot3(u, w) / (rij * rik);      /* edges i->j, i->k */
    double cos_j = dot3(mu, v) / (rij * rjk);     /* edges j->i, j->k */
    double cos_k = dot3(w, v) / (rik * rjk);      /* edges k->i = -w, k->j = -v */
    double prod = rij * rik * rjk;
    return nu * (1.0 + 3.0 * cos_i * cos_j * cos_k) / (prod * prod * prod);
}

/* ATM forces as -grad(phi3) written through the squared edge lengths a = |u|^2,
 * b = |w|^2, c = |v|^2.  By the law of cosines the cosine product equals
 * t1 t2 t3 / (8 a b c) with t1 = a+b-c, t2 = a-b+c, t3 = -a+b+c, so
 *   phi3 = nu [ P^(-3/2) + (3/8) T P^(-5/2) ],  P = a b c,  T = t1 t2 t3.
 * Differentiating (dP/da = P/a, dT/da = 2a t3 - t1 t2, and cyclically):
 *   phi_a = nu [ K/a + (3/8) P^(-5/2) (2a t3 - t1 t2) ]
 *   phi_b = nu [ K/b + (3/8) P^(-5/2) (2b t2 - t1 t3) ]
 *   phi_c = nu [ K/c + (3/8) P^(-5/2) (2c t1 - t2 t3) ]
 *   K     = -(3/2) P^(-3/2) - (15/16) T P^(-5/2).
 * With da/dx_j = 2u = -da/dx_i, db/dx_k = 2w = -db/dx_i, dc/dx_k = 2v = -dc/dx_j:
 *   F_i =  2 phi_a u + 2 phi_b w,  F_j = -2 phi_a u + 2 phi_c v,  F_k = -2 phi_b w - 2 phi_c v. */
static void atm_forces(const double *u, const double *w, const double *v, double nu,
                       double fi[3], double fj[3], double fk[3]) {
    double a = dot3(u, u), b = dot3(w, w), c = dot3(v, v);
    double P = a * b * c;
    double t1 = a + b - c, t2 = a - b + c, t3 = -a + b + c;
    double T = t1 * t2 * t3;
    double p32 = 1.0 / (P * sqrt(P));
    double p52 = p32 / P;
    double K = -1.5 * p32 - (15.0 / 16.0) * T * p52;
    double pa = nu * (K / a + 0.375 * p52 * (2.0 * a * t3 - t1 * t2));
    double pb = nu * (K / b + 0.375 * p52 * (2.0 * b * t2 - t1 * t3));
    double pc = nu * (K / c + 0.375 * p52 * (2.0 * c * t1 - t2 * t3));
    for (int d = 0; d < 3; ++d) {
        fi[d] = 2.0 * pa * u[d] + 2.0 * pb * w[d];
        fj[d] = -2.0 * pa * u[d] + 2.0 * pc * v[d];
        fk[d] = -2.0 * pb * w[d] - 2.0 * pc * v[d];
    }
}

/* Does the triplet (i, j, k) interact?  u, w, v are filled with the minimum-image
 * displacements i->j, i->k, j->k.  All three squared lengths must be <= rc2, and the
 * three images must close the triangle (u + v - w = 0 up to rounding). */
static int triplet_in(const double *xi, const double *xj, const double *xk, const double *L,
                      double rc2, double u[3], double w[3], double v[3]) {
    if (disp2(xi, xj, L, u) > rc2) return 0;
    if (disp2(xi, xk, L, w) > rc2) return 0;
    if (disp2(xj, xk, L, v) > rc2) return 0;
    for (int c = 0; c < 3; ++c)
        if (fabs(u[c] + v[c] - w[c]) >= 0.5 * L[c]) return 0;
    return 1;
}

static int all_finite(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int nthreads_of(int req) {
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* ------------------------------------------------------------------ pair forces */

/* F2 for all particles (O(N^2), i<j), energy U2 (optionally shifted), virial W2 and
 * the number of interacting pairs.  uw = {U2, W2}. */
int orc_pair(int64_t n, const double *x, const double *L, double eps, double sigma, double rc,
             int shift, double *f, double *uw, int64_t *npairs, int nthreads) {
    if (n < 0 || rc <= 0.0) return ORC_ERR_INVALID_ARG;
    if (!box_ok(L, rc)) return ORC_ERR_BOX_TOO_SMALL;
    double *xw = wrapped_copy(n, x, L);
    if (!xw) return ORC_ERR_OOM;
    int nt = nthreads_of(nthreads);
    double *fp = (double *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1) * 3, sizeof(double));
    double *ue = (double *)calloc((size_t)nt * 2, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    if (!fp || !ue || !cnt) { free(xw); free(fp); free(ue); free(cnt); return ORC_ERR_OOM; }
    double rc2 = rc * rc, dummy;
    double ushift = shift ? lj(rc2, eps, sigma, &dummy) : 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static, 8) num_threads(nt)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *ft = fp + (size_t)t * (size_t)n * 3;
        for (int64_t j = i + 1; j < n; ++j) {
            double d[3];
            double r2 = disp2(xw + 3 * i, xw + 3 * j, L, d);
            if (r2 > rc2) continue;
            double fr;
            double e = lj(r2, eps, sigma, &fr);
            for (int c = 0; c < 3; ++c) {
                ft[3 * j + c] += fr * d[c];
                ft[3 * i + c] -= fr * d[c];
            }
            ue[2 * t] += e - ushift;
            ue[2 * t + 1] += fr * r2;
            cnt[t] += 1;
        }
    }
    memset(f, 0, (size_t)n * 3 * sizeof(double));
    uw[0] = uw[1] = 0.0;
    int64_t np = 0;
    for (int t = 0; t < nt; ++t) {
        for (int64_t q = 0; q < 3 * n; ++q) f[q] += fp[(size_t)t * (size_t)n * 3 + q];
        uw[0] += ue[2 * t];
        uw[1] += ue[2 * t + 1];
        np += cnt[t];
    }
    if (npairs) *npairs = np;
    free(xw); free(fp); free(ue); free(cnt);
    if (!all_finite(f, 3 * n) || !all_finite(uw, 2)) return ORC_ERR_NONFINITE;
    return ORC_OK;
}

/* ------------------------------------------------------------------ triplet forces */

/* F3 for all particles by pruned brute force: loop i<j, skip k when (i,j) is out of
 * range, loop k>j.  uw = {U3, W3}; W3 sums x_a . F_a over the three members, written
 * relative to particle i as u . F_j + w . F_k.
 * Distance class (the intermediate cutoffs of Sec. 5, after the related work of Sec. 3):
 * with r_lo > 0 a triplet of T(rc) counts only if its longest edge exceeds r_lo, i.e.
 * unless all three squared edges are <= r_lo^2.  Classes (0, ra] and (ra, rc] thus
 * split T(rc) into two disjoint parts; r_lo <= 0 keeps all of T(rc). */
int orc_triplet_class(int64_t n, const double *x, const double *L, double nu, double r_lo,
                      double rc, double *f, double *uw, int64_t *ntrip, int nthreads) {
    if (n < 0 || rc <= 0.0) return ORC_ERR_INVALID_ARG;
    if (!box_ok(L, rc)) return ORC_ERR_BOX_TOO_SMALL;
    double *xw = wrapped_copy(n, x, L);
    if (!xw) return ORC_ERR_OOM;
    int nt = nthreads_of(nthreads);
    double *fp = (double *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1) * 3, sizeof(double));
    double *ue = (double *)calloc((size_t)nt * 2, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    if (!fp || !ue || !cnt) { free(xw); free(fp); free(ue); free(cnt); return ORC_ERR_OOM; }
    double rc2 = rc * rc;
    double lo2 = r_lo > 0.0 ? r_lo * r_lo : -1.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static, 4) num_threads(nt)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *ft = fp + (size_t)t * (size_t)n * 3;
        for (int64_t j = i + 1; j < n; ++j) {
            double u[3];
            if (disp2(xw + 3 * i, xw + 3 * j, L, u) > rc2) continue;
            for (int64_t k = j + 1; k < n; ++k) {
                double w[3], v[3];
                if (!triplet_in(xw + 3 * i, xw + 3 * j, xw + 3 * k, L, rc2, u, w, v)) continue;
                if (dot3(u, u) <= lo2 && dot3(w, w) <= lo2 && dot3(v, v) <= lo2) continue;
                double fi[3], fj[3], fk[3];
                atm_forces(u, w, v, nu, fi, fj, fk);
                for (int c = 0; c < 3; ++c) {
                    ft[3 * i + c] += fi[c];
                    ft[3 * j + c] += fj[c];
                    ft[3 * k + c] += fk[c];
                }
                ue[2 * t] += atm_energy(u, w, v, nu);
                ue[2 * t + 1] += dot3(u, fj) + dot3(w, fk);
                cnt[t] += 1;
            }
        }
    }
    memset(f, 0, (size_t)n * 3 * sizeof(double));
    uw[0] = uw[1] = 0.0;
    int64_t nn = 0;
    for (int t = 0; t < nt; ++t) {
        for (int64_t q = 0; q < 3 * n; ++q) f[q] += fp[(size_t)t * (size_t)n * 3 + q];
        uw[0] += ue[2 * t];
        uw[1] += ue[2 * t + 1];
        nn += cnt[t];
    }
    if (ntrip) *ntrip = nn;
    free(xw); free(fp); free(ue); free(cnt);
    if (!all_finite(f, 3 * n) || !all_finite(uw, 2)) return ORC_ERR_NONFINITE;
    return ORC_OK;
}

int orc_triplet(int64_t n, const double *x, const double *L, double nu, double rc, double *f,
                double *uw, int64_t *ntrip, int nthreads) {
    return orc_triplet_class(n, x, L, nu, 0.0, rc, f, uw, ntrip, nthreads);
}

/* Every interacting triplet as (i, j, k), i<j<k, in lexicographic order.  Returns the
 * total count (which may exceed cap; only the first cap are written), or < 0 on error. */
int64_t orc_triplet_list(int64_t n, const double *x, const double *L, double rc, int32_t *ijk,
                         int64_t cap) {
    if (n < 0 || rc <= 0.0) return ORC_ERR_INVALID_ARG;
    if (!box_ok(L, rc)) return ORC_ERR_BOX_TOO_SMALL;
    double *xw = wrapped_copy(n, x, L);
    if (!xw) return ORC_ERR_OOM;
    double rc2 = rc * rc;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double u[3];
            if (disp2(xw + 3 * i, xw + 3 * j, L, u) > rc2) continue;
            for (int64_t k = j + 1; k < n; ++k) {
                double w[3], v[3];
                if (!triplet_in(xw + 3 * i, xw + 3 * j, xw + 3 * k, L, rc2, u, w, v)) continue;
                if (cnt < cap) {
                    ijk[3 * cnt] = (int32_t)i;
                    ijk[3 * cnt + 1] = (int32_t)j;
                    ijk[3 * cnt + 2] = (int32_t)k;
                }
                ++cnt;
            }
        }
    free(xw);
    return cnt;
}

/* Exact F2 and F3 on a subset of particles of an arbitrarily large system: for each
 * chosen particle p, scan all N particles for its neighbours and sum every pair and
 * every triplet that contains p (p plays the role of i in the formulas above).
 * counts (nullable) receives {pairs, triplets} summed over the chosen particles: a pair
 * or triplet holding two or three of them is counted once per chosen member. */
int orc_subset(int64_t n, const double *x, const double *L, double eps, double sigma,
               double rc_pair, double nu, double rc3, int64_t ns, const int64_t *idx,
               double *f2, double *f3, int64_t *counts, int nthreads) {
    if (n < 0 || ns < 0 || rc_pair <= 0.0 || rc3 <= 0.0) return ORC_ERR_INVALID_ARG;
    if (!box_ok(L, rc_pair) || !box_ok(L, rc3)) return ORC_ERR_BOX_TOO_SMALL;
    for (int64_t s = 0; s < ns; ++s)
        if (idx[s] < 0 || idx[s] >= n) return ORC_ERR_INVALID_ARG;
    double *xw = wrapped_copy(n, x, L);
    if (!xw) return ORC_ERR_OOM;
    double rcp2 = rc_pair * rc_pair, rc32 = rc3 * rc3;
    int nt = nthreads_of(nthreads);
    int failed = 0;
    int64_t npair = 0, ntrip = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(+ : npair, ntrip)
#endif
    for (int64_t s = 0; s < ns; ++s) {
        int64_t p = idx[s];
        int64_t cap = 256, m = 0;
        int64_t *nb = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
        double fp2[3] = {0, 0, 0}, fp3[3] = {0, 0, 0};
        if (!nb) { failed = 1; continue; }
        for (int64_t q = 0; q < n; ++q) {
            if (q == p) continue;
            double d[3];
            double r2 = disp2(xw + 3 * p, xw + 3 * q, L, d);
            if (r2 <= rcp2) {
                double fr;
                (void)lj(r2, eps, sigma, &fr);
                for (int c = 0; c < 3; ++c) fp2[c] -= fr * d[c];
                ++npair;
            }
            if (r2 <= rc32) {
                if (m == cap) {
                    cap *= 2;
                    int64_t *nn = (int64_t *)realloc(nb, (size_t)cap * sizeof(int64_t));
                    if (!nn) { failed = 1; break; }
                    nb = nn;
                }
                nb[m++] = q;
            }
        }
        for (int64_t a = 0; a < m; ++a)
            for (int64_t b = a + 1; b < m; ++b) {
                double u[3], w[3], v[3], fi[3], fj[3], fk[3];
                if (!triplet_in(xw + 3 * p, xw + 3 * nb[a], xw + 3 * nb[b], L, rc32, u, w, v))
                    continue;
                atm_forces(u, w, v, nu, fi, fj, fk);
                for (int c = 0; c < 3; ++c) fp3[c] += fi[c];
                ++ntrip;
            }
        for (int c = 0; c < 3; ++c) {
            f2[3 * s + c] = fp2[c];
            f3[3 * s + c] = fp3[c];
        }
        free(nb);
    }
    free(xw);
    if (failed) return ORC_ERR_OOM;
    if (counts) {
        counts[0] = npair;
        counts[1] = ntrip;
    }
    if (!all_finite(f2, 3 * ns) || !all_finite(f3, 3 * ns)) return ORC_ERR_NONFINITE;
    return ORC_OK;
}

/* ------------------------------------------------------------------ integrators */

typedef struct {
    double eps, sigma, rc_pair, nu, rc3, mass, dt;
    int shift, nthreads;
} orc_md;

static double kinetic(int64_t n, const double *v, double m) {
    double s = 0.0;
    for (int64_t q = 0; q < 3 * n; ++q) s += v[q] * v[q];
    return 0.5 * m * s;
}

/* e = {K, U2, U3, W2, W3} */
static void record(double *e, double K, const double *uw2, const double *uw3) {
    e[0] = K;
    e[1] = uw2[0];
    e[2] = uw3[0];
    e[3] = uw2[1];
    e[4] = uw3[1];
}

/* v <- v + c f, element by element. */
static void kick(int64_t n, double *v, const double *f, double c) {
    for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q] + c * f[q];
}

/* One velocity-Verlet step of length h on the pair force alone, with the velocity
 * half-kicks of the step merged: the drift x <- wrap(x + h v + h^2/(2m) F2(x)), then the
 * new pair force and v <- v + h/(2m) (F2(x_old) + F2(x_new)).  *f2 holds F2(x) on entry
 * and F2(x_new) on exit (the two buffers are swapped); uw2 gets {U2, W2} at x_new. */
static int vv_pair_step(int64_t n, double *x, double *v, const double *L, const orc_md *p,
                        double h, double **f2, double **f2n, double uw2[2]) {
    const double cx = (h * h) / (2.0 * p->mass);
    const double c2 = h / (2.0 * p->mass);
    double *fo = *f2, *fn = *f2n;
    for (int64_t a = 0; a < n; ++a)
        for (int d = 0; d < 3; ++d) {
            int64_t q = 3 * a + d;
            x[q] = wrap1(x[q] + h * v[q] + cx * fo[q], L[d]);
        }
    int rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, fn, uw2, NULL, p->nthreads);
    if (rc != ORC_OK) return rc;
    for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q] + c2 * (fo[q] + fn[q]);
    *f2 = fn;
    *f2n = fo;
    return ORC_OK;
}

/* r-RESPA as the paper runs it (Sec. 4.1, Algorithm 2) with step-size factor s = k: the
 * three-body force acts as an impulse of half an outer step (dt k) at each end of an
 * outer cycle, and the pair force moves the particles through the k inner steps of
 * velocity Verlet between the two impulses.  Only the ends of the cycles are full steps,
 * where velocities are synchronised; e_full holds {K,U2,U3,W2,W3} at x^0 and after each
 * cycle: n_iter/k + 1 rows.  x and v are updated in place. */
int orc_respa(int64_t n, double *x, double *v, const double *L, const orc_md *p, int64_t n_iter,
              int k, double *e_full) {
    if (n < 0 || n_iter < 0 || k < 1 || p->dt <= 0.0 || p->mass <= 0.0) return ORC_ERR_INVALID_ARG;
    if (n_iter % k != 0) return ORC_ERR_NOT_MULTIPLE_OF_K;
    size_t bytes = (size_t)(n > 0 ? n : 1) * 3 * sizeof(double);
    double *b2 = (double *)malloc(bytes), *b2n = (double *)malloc(bytes), *f3 = (double *)malloc(bytes);
    if (!b2 || !b2n || !f3) { free(b2); free(b2n); free(f3); return ORC_ERR_OOM; }
    double *f2 = b2, *f2n = b2n;
    double uw2[2], uw3[2];
    int rc;
    rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, f2, uw2, NULL, p->nthreads);
    if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f3, uw3, NULL, p->nthreads);
    if (rc == ORC_OK && e_full) record(e_full, kinetic(n, v, p->mass), uw2, uw3);
    const double impulse = (p->dt * (double)k) / (2.0 * p->mass);  /* half an outer step */
    for (int64_t cyc = 0; rc == ORC_OK && cyc < n_iter / k; ++cyc) {
        kick(n, v, f3, impulse);
        for (int s = 0; rc == ORC_OK && s < k; ++s)
            rc = vv_pair_step(n, x, v, L, p, p->dt, &f2, &f2n, uw2);
        if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f3, uw3, NULL, p->nthreads);
        if (rc != ORC_OK) break;
        kick(n, v, f3, impulse);
        if (e_full) record(e_full + 5 * (cyc + 1), kinetic(n, v, p->mass), uw2, uw3);
    }
    free(b2); free(b2n); free(f3);
    return rc;
}

/* The two distance classes of T(rc3) split at r_a: inner (longest edge <= r_a) into fin,
 * outer (r_a < longest edge <= rc3) into fout; uw gets {U, W} of both classes summed.
 * r_a == 0: the inner class is empty; r_a >= rc3: the outer class is empty. */
static int class_forces(int64_t n, const double *x, const double *L, const orc_md *p, double r_a,
                        double *fin, double *fout, double uw[2], int want_in, int want_out) {
    double ui[2] = {0.0, 0.0}, uo[2] = {0.0, 0.0};
    int rc = ORC_OK;
    if (want_in) {
        if (r_a > 0.0)
            rc = orc_triplet_class(n, x, L, p->nu, 0.0, r_a < p->rc3 ? r_a : p->rc3, fin, ui, NULL,
                                   p->nthreads);
        else
            memset(fin, 0, (size_t)n * 3 * sizeof(double));
    }
    if (rc == ORC_OK && want_out) {
        if (r_a < p->rc3)
            rc = orc_triplet_class(n, x, L, p->nu, r_a, p->rc3, fout, uo, NULL, p->nthreads);
        else
            memset(fout, 0, (size_t)n * 3 * sizeof(double));
    }
    uw[0] = ui[0] + uo[0];
    uw[1] = ui[1] + uo[1];
    return rc;
}

/* r-RESPA with three time scales: the nested form of Sec. 2.3.1 (one more level, as the
 * text allows for any number of force splittings) over the triplet distance classes of
 * Sec. 5.  F2 drives velocity Verlet with the inner step dt; the inner triplet class Fin
 * acts as impulses of half of k inner steps around every group of k inner steps, the
 * outer class Fout as impulses of half of k k_outer inner steps around every k_outer such
 * groups (an outer cycle).  Velocities are synchronised only at the ends of outer cycles:
 * e_full holds {K, U2, U3, W2, W3} (U3, W3 over both classes) at x^0 and after every
 * outer cycle: n_iter / (k k_outer) + 1 rows.  k_outer = 1 is Algorithm 2 with s = k. */
int orc_respa_nested(int64_t n, double *x, double *v, const double *L, const orc_md *p,
                     int64_t n_iter, int k, int k_outer, double r_a, double *e_full) {
    if (n < 0 || n_iter < 0 || k < 1 || k_outer < 1 || r_a < 0.0 || p->dt <= 0.0 ||
        p->mass <= 0.0)
        return ORC_ERR_INVALID_ARG;
    const int64_t span = (int64_t)k * (int64_t)k_outer;
    if (n_iter % span != 0) return ORC_ERR_NOT_MULTIPLE_OF_K;
    size_t bytes = (size_t)(n > 0 ? n : 1) * 3 * sizeof(double);
    double *b2 = (double *)malloc(bytes), *b2n = (double *)malloc(bytes);
    double *fin = (double *)malloc(bytes), *fout = (double *)malloc(bytes);
    if (!b2 || !b2n || !fin || !fout) {
        free(b2); free(b2n); free(fin); free(fout);
        return ORC_ERR_OOM;
    }
    double *f2 = b2, *f2n = b2n;
    double uw2[2], uw3[2];
    int rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, f2, uw2, NULL, p->nthreads);
    if (rc == ORC_OK) rc = class_forces(n, x, L, p, r_a, fin, fout, uw3, 1, 1);
    if (rc == ORC_OK && e_full) record(e_full, kinetic(n, v, p->mass), uw2, uw3);
    const double imp_in = (p->dt * (double)k) / (2.0 * p->mass);
    const double imp_out = (p->dt * (double)span) / (2.0 * p->mass);
    double uin[2], uout[2];
    for (int64_t cyc = 0; rc == ORC_OK && cyc < n_iter / span; ++cyc) {
        kick(n, v, fout, imp_out);
        for (int g = 0; rc == ORC_OK && g < k_outer; ++g) {
            kick(n, v, fin, imp_in);
            for (int s = 0; rc == ORC_OK && s < k; ++s)
                rc = vv_pair_step(n, x, v, L, p, p->dt, &f2, &f2n, uw2);
            if (rc == ORC_OK) rc = class_forces(n, x, L, p, r_a, fin, fout, uin, 1, 0);
            if (rc == ORC_OK) kick(n, v, fin, imp_in);
        }
        if (rc == ORC_OK) rc = class_forces(n, x, L, p, r_a, fin, fout, uout, 0, 1);
        if (rc != ORC_OK) break;
        uw3[0] = uin[0] + uout[0];  /* uin: the inner class at this same x, just computed */
        uw3[1] = uin[1] + uout[1];
        kick(n, v, fout, imp_out);
        if (e_full) record(e_full + 5 * (cyc + 1), kinetic(n, v, p->mass), uw2, uw3);
    }
    free(b2); free(b2n); free(fin); free(fout);
    return rc;
}

/* Algorithm 1 (Sec. 2.3.1) with the fast force F0 = F2 and the slow force F1 = F3:
 * p->dt is the full step delta t, split into P sub-steps h = delta t / P.  The slow
 * force acts as impulses of delta t / 2 at both ends of every full step, the fast one
 * moves the particles through P velocity-Verlet sub-steps of length h in between.
 * Readings of the garbled parts: the sub-step velocity update adds h/(2m) times the sum
 * of the fast force at the sub-step's two ends, and the closing impulse uses delta t.
 * e holds {K,U2,U3,W2,W3} at x^0 and after every full step: n_outer + 1 rows. */
int orc_respa_alg1(int64_t n, double *x, double *v, const double *L, const orc_md *p,
                   int64_t n_outer, int P, double *e) {
    if (n < 0 || n_outer < 0 || P < 1 || p->dt <= 0.0 || p->mass <= 0.0) return ORC_ERR_INVALID_ARG;
    size_t bytes = (size_t)(n > 0 ? n : 1) * 3 * sizeof(double);
    double *b0 = (double *)malloc(bytes), *b0n = (double *)malloc(bytes), *f1 = (double *)malloc(bytes);
    if (!b0 || !b0n || !f1) { free(b0); free(b0n); free(f1); return ORC_ERR_OOM; }
    double *f0 = b0, *f0n = b0n;
    double uw2[2], uw3[2];
    int rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, f0, uw2, NULL, p->nthreads);
    if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f1, uw3, NULL, p->nthreads);
    if (rc == ORC_OK && e) record(e, kinetic(n, v, p->mass), uw2, uw3);
    const double h = p->dt / (double)P;
    const double impulse = p->dt / (2.0 * p->mass);
    for (int64_t i = 0; rc == ORC_OK && i < n_outer; ++i) {
        kick(n, v, f1, impulse);
        for (int j = 0; rc == ORC_OK && j < P; ++j)
            rc = vv_pair_step(n, x, v, L, p, h, &f0, &f0n, uw2);
        if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f1, uw3, NULL, p->nthreads);
        if (rc != ORC_OK) break;
        kick(n, v, f1, impulse);
        if (e) record(e + 5 * (i + 1), kinetic(n, v, p->mass), uw2, uw3);
    }
    free(b0); free(b0n); free(f1);
    return rc;
}

/* Textbook velocity Verlet with the total force F = F2 + F3 every step:
 *   v_half = v + (dt/2m) F(x);  x <- x + dt v_half;  v = v_half + (dt/2m) F(x_new).
 * e holds {K,U2,U3,W2,W3} at x^0 and after every step: n_iter + 1 rows. */
int orc_vv(int64_t n, double *x, double *v, const double *L, const orc_md *p, int64_t n_iter,
           double *e) {
    if (n < 0 || n_iter < 0 || p->dt <= 0.0 || p->mass <= 0.0) return ORC_ERR_INVALID_ARG;
    size_t bytes = (size_t)(n > 0 ? n : 1) * 3 * sizeof(double);
    double *f2 = (double *)malloc(bytes), *f3 = (double *)malloc(bytes);
    if (!f2 || !f3) { free(f2); free(f3); return ORC_ERR_OOM; }
    double uw2[2], uw3[2];
    int rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, f2, uw2, NULL, p->nthreads);
    if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f3, uw3, NULL, p->nthreads);
    if (rc != ORC_OK) { free(f2); free(f3); return rc; }
    if (e) record(e, kinetic(n, v, p->mass), uw2, uw3);
    const double h = p->dt / (2.0 * p->mass);
    for (int64_t s = 0; s < n_iter; ++s) {
        for (int64_t a = 0; a < n; ++a)
            for (int c = 0; c < 3; ++c) {
                int64_t q = 3 * a + c;
                double vh = v[q] + h * (f2[q] + f3[q]);
                v[q] = vh;
                x[q] = wrap1(x[q] + p->dt * vh, L[c]);
            }
        rc = orc_pair(n, x, L, p->eps, p->sigma, p->rc_pair, p->shift, f2, uw2, NULL, p->nthreads);
        if (rc == ORC_OK) rc = orc_triplet(n, x, L, p->nu, p->rc3, f3, uw3, NULL, p->nthreads);
        if (rc != ORC_OK) break;
        for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q] + h * (f2[q] + f3[q]);
        if (e) record(e + 5 * (s + 1), kinetic(n, v, p->mass), uw2, uw3);
    }
    free(f2); free(f3);
    return rc;
}

/* Single-triplet and single-pair evaluations for closed-form checks. */
double orc_atm_energy(const double *u, const double *w, double nu) {
    double v[3] = {w[0] - u[0], w[1] - u[1], w[2] - u[2]};
    return atm_energy(u, w, v, nu);
}

void orc_atm_forces(const double *u, const double *w, double nu, double *fijk) {
    double v[3] = {w[0] - u[0], w[1] - u[1], w[2] - u[2]};
    atm_forces(u, w, v, nu, fijk, fijk + 3, fijk + 6);
}

double orc_lj(double r2, double eps, double sigma, double *fr) { return lj(r2, eps, sigma, fr); }
