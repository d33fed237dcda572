/*
 * Plain FP64 CPU oracle for the adaptive-resolution weakly-compressible SPH
 * hot path of Muta & Ramachandran, "Efficient and accurate adaptive
 * resolution for weakly-compressible SPH" (arXiv 2107.01276).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  It shares no code,
 * header, table or constant generator with the HIP library; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * Nothing on the product path may call it.
 *
 * Conventions (each function cites the passage it follows):
 *   - all arithmetic in double precision, built with -ffp-contract=off and
 *     no fast-math, so every operation is rounded once, in program order;
 *   - every pair sum runs over a neighbour row in ascending particle index;
 *   - updates are Jacobi: new values are written to separate arrays and
 *     applied after the loop.
 *
 * Readings where the paper is silent or garbled are marked READING and are
 * listed in the design notes of the repository.
 *
 * Parity pins: every public function is pinned by tests against brute force,
 * closed forms, invariants or values printed in the paper, except where its
 * comment says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Public structs (mirrored by ctypes in oracle/__init__.py).                */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[2];
    double hi[2];
    int32_t periodic[2];
} or_domain;

typedef struct {
    double rho0;        /* reference density rho_0 */
    double cs;          /* artificial speed of sound c_s */
    double nu;          /* kinematic viscosity */
    double alpha_e;     /* EDAC viscosity factor (1.5 in the paper) */
    double hdx;         /* h / dx, the constant C of h = C (m/rho)^(1/d) */
    double fx, fy;      /* body force */
    double split_alpha; /* child h factor (0.9) */
    double split_eps;   /* child radius factor (0.4) */
    double mmax_f;      /* m_max = mmax_f * m_ref (1.05) */
    double mmin_f;      /* m_min = mmin_f * m_ref (0.5), reported only */
    double mass_q;      /* mass quantum: m = mq * mass_q exactly */
    int32_t merge_iters;
    int32_t shift_iters;
    int32_t pref_mode;  /* READING, pressure reduction of eq. (mom:pre):
                           1 (used): both P_i and P_j subtract p_avg,i, the
                           average over particle i's neighbourhood;
                           0: P_j subtracts p_avg,j as printed, which cancels
                           the force of any linear pressure field and fails
                           the Taylor-Green exact solution of section 4.1. */
} or_params;

typedef struct {
    double rho0;
    double cr;          /* size ratio between adjacent background layers */
    double ds_min, ds_max;
    double n_r;         /* reference neighbour count (48) */
    double split_alpha, split_eps, mmax_f;
    double mass_q;      /* mass quantum of the background ledger */
    int32_t smooth_iters; /* h-smoothing + PST repetitions (3) */
} or_bgparams;

#define OR_OK 0
#define OR_E_CAPACITY (-2)
#define OR_E_NOMEM (-3)
#define OR_E_INVAL (-1)

/* ------------------------------------------------------------------------ */
/* Quintic spline kernel, eq. (kernel), section 2.                           */
/* W(r,h) = sigma2(h) f(q), q = r/h, sigma2 = 7 / (478 pi h^2).              */
/* ------------------------------------------------------------------------ */

static const double OR_SIGMA = 0.00466144184787978; /* 7 / (478 pi) */
static const double OR_XI = 0.759298480738450;     /* inflection point, sec. 2.1 */
static const double OR_SIN60 = 0.8660254037844386; /* sin(pi/3) */

static double qpow5(double a) { double a2 = a * a; return a2 * a2 * a; }
static double qpow4(double a) { double a2 = a * a; return a2 * a2; }

/* f(q): the bracketed polynomial of eq. (kernel). */
double or_kf(double q)
{
    if (q >= 3.0) return 0.0;
    double v = qpow5(3.0 - q);
    if (q < 2.0) v = v - 6.0 * qpow5(2.0 - q);
    if (q < 1.0) v = v + 15.0 * qpow5(1.0 - q);
    return v;
}

/* df/dq. */
double or_kfp(double q)
{
    if (q >= 3.0) return 0.0;
    double v = -5.0 * qpow4(3.0 - q);
    if (q < 2.0) v = v + 30.0 * qpow4(2.0 - q);
    if (q < 1.0) v = v - 75.0 * qpow4(1.0 - q);
    return v;
}

double or_w(double r, double h)
{
    double q = r / h;
    return (OR_SIGMA / (h * h)) * or_kf(q);
}

/* dW/dr = sigma2(h) f'(q) / h. */
double or_dwdr(double r, double h)
{
    double q = r / h;
    return (OR_SIGMA / (h * h)) * or_kfp(q) / h;
}

/* ------------------------------------------------------------------------ */
/* Geometry: minimum-image displacement r_i - r_j and periodic wrapping.     */
/* READING: a displacement of exactly half the period is not wrapped.        */
/* ------------------------------------------------------------------------ */

static double mi_axis(const or_domain* d, int a, double dx)
{
    if (d->periodic[a]) {
        double L = d->hi[a] - d->lo[a];
        double half = 0.5 * L;
        if (dx > half) dx = dx - L;
        else if (dx < -half) dx = dx + L;
    }
    return dx;
}

static double wrap_axis(const or_domain* d, int a, double x)
{
    if (d->periodic[a]) {
        double L = d->hi[a] - d->lo[a];
        if (x < d->lo[a]) x = x + L;
        else if (x >= d->hi[a]) x = x - L;
        if (x >= d->hi[a] || x < d->lo[a]) x = d->lo[a];
    }
    return x;
}

/* Neighbour predicate: j in N(i) iff |r_ij|^2 < (3 max(h_i,h_j))^2, with the
 * squared distance dx*dx + dy*dy (READING: symmetric support, strict, self
 * included; the rates of eq. (edac:sph) and eq. (mom-sph) use both W(h_i) and
 * W(h_j), so a pair interacts when either support covers it). */
static int is_nbr(const or_domain* d, double xi, double yi, double hi_,
                  double xj, double yj, double hj)
{
    double dx = mi_axis(d, 0, xi - xj);
    double dy = mi_axis(d, 1, yi - yj);
    double r2 = dx * dx + dy * dy;
    double hm = hi_ > hj ? hi_ : hj;
    double R = 3.0 * hm;
    return r2 < R * R;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists as CSR: row_ptr[n+1] (int64), col[nnz] (int32), rows in  */
/* ascending column order, self included.                                    */
/* ------------------------------------------------------------------------ */

/* Brute force O(n^2).  Returns nnz; col is written only if nnz <= cap. */
int64_t or_nbr_brute(const or_domain* d, int64_t n, const double* x,
                     const double* y, const double* h, int64_t* row_ptr,
                     int32_t* col, int64_t cap)
{
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            c += is_nbr(d, x[i], y[i], h[i], x[j], y[j], h[j]);
        row_ptr[i + 1] = row_ptr[i] + c;
    }
    int64_t nnz = row_ptr[n];
    if (nnz > cap) return nnz;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = row_ptr[i];
        for (int64_t j = 0; j < n; ++j)
            if (is_nbr(d, x[i], y[i], h[i], x[j], y[j], h[j])) col[k++] = (int32_t)j;
    }
    return nnz;
}

/* Brute-force cross query: rows over set A, columns index set B, same
 * predicate with max(h_a, h_b). */
int64_t or_xnbr_brute(const or_domain* d, int64_t na, const double* xa,
                      const double* ya, const double* ha, int64_t nb,
                      const double* xb, const double* yb, const double* hb,
                      int64_t* row_ptr, int32_t* col, int64_t cap)
{
    row_ptr[0] = 0;
    for (int64_t i = 0; i < na; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < nb; ++j)
            c += is_nbr(d, xa[i], ya[i], ha[i], xb[j], yb[j], hb[j]);
        row_ptr[i + 1] = row_ptr[i] + c;
    }
    int64_t nnz = row_ptr[na];
    if (nnz > cap) return nnz;
    for (int64_t i = 0; i < na; ++i) {
        int64_t k = row_ptr[i];
        for (int64_t j = 0; j < nb; ++j)
            if (is_nbr(d, xa[i], ya[i], ha[i], xb[j], yb[j], hb[j])) col[k++] = (int32_t)j;
    }
    return nnz;
}

/* Cell-list neighbour search, for sizes brute force cannot reach.  Plain
 * construction: particles are grouped by h level (powers of two above the
 * smallest h); each level has a uniform grid of cell width >= 3 hmax(level).
 * Every particle scans its own and every coarser level with search radius
 * 3 hmax(level), which covers 3 max(h_i, h_j) for every pair it can meet
 * there.  A pair across two levels is seen only from the finer particle, so
 * it is recorded in both directions; a pair within one level is seen from
 * both sides and recorded once per side.  Rows are then sorted. */

typedef struct {
    int64_t count;
    double hmax;
    double org[2], cw[2];
    int nc[2];
    int64_t* start; /* nc0*nc1 + 1 */
    int64_t* items;
} or_level;

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int axis_range(const or_domain* d, int a, double xi, double R,
                      double org, double cw, int nc, int* ks)
{
    double slack = 1e-9 * R + 1e-13 * (fabs(xi) + fabs(org) + cw * nc);
    double lo = floor((xi - R - slack - org) / cw);
    double hi = floor((xi + R + slack - org) / cw);
    int m = 0;
    if (d->periodic[a]) {
        if (hi - lo + 1.0 >= (double)nc) {
            for (int k = 0; k < nc; ++k) ks[m++] = k;
        } else {
            for (double k = lo; k <= hi; k += 1.0) {
                long kk = (long)k % nc;
                if (kk < 0) kk += nc;
                ks[m++] = (int)kk;
            }
        }
    } else {
        if (lo < 0) lo = 0;
        if (hi > nc - 1) hi = nc - 1;
        for (double k = lo; k <= hi; k += 1.0) ks[m++] = (int)k;
    }
    return m;
}

static int cell_of(const or_domain* d, int a, double xi, double org, double cw, int nc)
{
    (void)d;
    double k = floor((xi - org) / cw);
    if (k < 0) k = 0;
    if (k > nc - 1) k = nc - 1;
    return (int)k;
}

/* Builds CSR into freshly allocated arrays.  Returns nnz or a negative error. */
int64_t or_nbr_cells_alloc(const or_domain* d, int64_t n, const double* x,
                           const double* y, const double* h,
                           int64_t** row_ptr_out, int32_t** col_out)
{
    int64_t* rp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!rp) return OR_E_NOMEM;
    *row_ptr_out = rp;
    *col_out = NULL;
    if (n == 0) { *col_out = (int32_t*)malloc(sizeof(int32_t)); return 0; }

    double hmin = h[0];
    for (int64_t i = 1; i < n; ++i) if (h[i] < hmin) hmin = h[i];
    int* lev = (int*)malloc(sizeof(int) * (size_t)n);
    int nlev = 0;
    for (int64_t i = 0; i < n; ++i) {
        int e = 0;
        frexp(h[i] / hmin, &e); /* h/hmin = f 2^e, f in [0.5,1) */
        int l = e - 1;
        if (l < 0) l = 0;
        if (l > 60) l = 60;
        lev[i] = l;
        if (l + 1 > nlev) nlev = l + 1;
    }
    /* bounding box for non-periodic axes */
    double bmin[2], bmax[2];
    for (int a = 0; a < 2; ++a) {
        const double* c = a ? y : x;
        bmin[a] = bmax[a] = c[0];
        for (int64_t i = 1; i < n; ++i) {
            if (c[i] < bmin[a]) bmin[a] = c[i];
            if (c[i] > bmax[a]) bmax[a] = c[i];
        }
    }
    or_level* L = (or_level*)calloc((size_t)nlev, sizeof(or_level));
    for (int64_t i = 0; i < n; ++i) {
        or_level* lv = &L[lev[i]];
        if (lv->count == 0 || h[i] > lv->hmax) lv->hmax = h[i];
        lv->count++;
    }
    for (int l = 0; l < nlev; ++l) {
        or_level* lv = &L[l];
        if (!lv->count) continue;
        for (int a = 0; a < 2; ++a) {
            double c = 3.0 * lv->hmax;
            if (d->periodic[a]) {
                double P = d->hi[a] - d->lo[a];
                int nc = (int)floor(P / c);
                if (nc < 1) nc = 1;
                lv->org[a] = d->lo[a];
                lv->cw[a] = P / nc;
                lv->nc[a] = nc;
            } else {
                double span = bmax[a] - bmin[a];
                lv->org[a] = bmin[a];
                lv->cw[a] = c;
                lv->nc[a] = (int)floor(span / c) + 1;
            }
        }
        /* keep the table modest for very sparse levels */
        while ((double)lv->nc[0] * lv->nc[1] > 16.0 * lv->count + 1024.0) {
            for (int a = 0; a < 2; ++a) {
                if (d->periodic[a]) {
                    int nc = lv->nc[a] / 2;
                    if (nc < 1) nc = 1;
                    lv->cw[a] = (d->hi[a] - d->lo[a]) / nc;
                    lv->nc[a] = nc;
                } else {
                    lv->cw[a] *= 2.0;
                    lv->nc[a] = (int)floor((bmax[a] - bmin[a]) / lv->cw[a]) + 1;
                }
            }
        }
        int64_t ncell = (int64_t)lv->nc[0] * lv->nc[1];
        lv->start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
        lv->items = (int64_t*)malloc(sizeof(int64_t) * (size_t)lv->count);
    }
    /* counting sort of each level's members into its cells */
    int64_t* cellid = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        or_level* lv = &L[lev[i]];
        int cx = cell_of(d, 0, x[i], lv->org[0], lv->cw[0], lv->nc[0]);
        int cy = cell_of(d, 1, y[i], lv->org[1], lv->cw[1], lv->nc[1]);
        cellid[i] = (int64_t)cy * lv->nc[0] + cx;
        lv->start[cellid[i] + 1]++;
    }
    for (int l = 0; l < nlev; ++l) {
        or_level* lv = &L[l];
        if (!lv->count) continue;
        int64_t ncell = (int64_t)lv->nc[0] * lv->nc[1];
        for (int64_t c = 0; c < ncell; ++c) lv->start[c + 1] += lv->start[c];
    }
    {
        int64_t** fill = (int64_t**)calloc((size_t)nlev, sizeof(int64_t*));
        for (int l = 0; l < nlev; ++l) {
            if (!L[l].count) continue;
            int64_t ncell = (int64_t)L[l].nc[0] * L[l].nc[1];
            fill[l] = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
            memcpy(fill[l], L[l].start, sizeof(int64_t) * (size_t)ncell);
        }
        for (int64_t i = 0; i < n; ++i) {
            or_level* lv = &L[lev[i]];
            lv->items[fill[lev[i]][cellid[i]]++] = i;
        }
        for (int l = 0; l < nlev; ++l) free(fill[l]);
        free(fill);
    }
    free(cellid);

    /* pair emission: pass 0 counts per row, pass 1 writes.  Rows are shared
     * (a pair found from the finer side is written to both rows), so the
     * threads bump the counts and fill cursors atomically; the order within
     * a row is then arbitrary and every row is sorted at the end. */
    int32_t* col = NULL;
    int64_t* fillp = NULL;
    int maxk = 0;
    for (int l = 0; l < nlev; ++l)
        for (int a = 0; a < 2; ++a) if (L[l].nc[a] > maxk) maxk = L[l].nc[a];
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
            col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
            fillp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
            for (int64_t i = 0; i < n; ++i) fillp[i] = rp[i];
        }
#pragma omp parallel
        {
        int* kx = (int*)malloc(sizeof(int) * (size_t)(maxk + 8));
        int* ky = (int*)malloc(sizeof(int) * (size_t)(maxk + 8));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            for (int l = lev[i]; l < nlev; ++l) {
                or_level* lv = &L[l];
                if (!lv->count) continue;
                double R = 3.0 * lv->hmax;
                int mx = axis_range(d, 0, x[i], R, lv->org[0], lv->cw[0], lv->nc[0], kx);
                int my = axis_range(d, 1, y[i], R, lv->org[1], lv->cw[1], lv->nc[1], ky);
                for (int b = 0; b < my; ++b)
                    for (int a = 0; a < mx; ++a) {
                        int64_t c = (int64_t)ky[b] * lv->nc[0] + kx[a];
                        for (int64_t t = lv->start[c]; t < lv->start[c + 1]; ++t) {
                            int64_t j = lv->items[t];
                            if (!is_nbr(d, x[i], y[i], h[i], x[j], y[j], h[j])) continue;
                            if (pass == 0) {
#pragma omp atomic
                                rp[i + 1]++;
                                if (l != lev[i]) {
#pragma omp atomic
                                    rp[j + 1]++;
                                }
                            } else {
                                int64_t at;
#pragma omp atomic capture
                                at = fillp[i]++;
                                col[at] = (int32_t)j;
                                if (l != lev[i]) {
#pragma omp atomic capture
                                    at = fillp[j]++;
                                    col[at] = (int32_t)i;
                                }
                            }
                        }
                    }
            }
        }
        free(kx);
        free(ky);
        }
    }
    free(fillp);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        qsort(col + rp[i], (size_t)(rp[i + 1] - rp[i]), sizeof(int32_t), cmp_i32);
    for (int l = 0; l < nlev; ++l) { free(L[l].start); free(L[l].items); }
    free(L);
    free(lev);
    *col_out = col;
    return rp[n];
}

/* Same as or_nbr_cells_alloc but into caller arrays (col written if nnz<=cap). */
int64_t or_nbr_cells(const or_domain* d, int64_t n, const double* x,
                     const double* y, const double* h, int64_t* row_ptr,
                     int32_t* col, int64_t cap)
{
    int64_t* rp = NULL;
    int32_t* c = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, x, y, h, &rp, &c);
    if (nnz < 0) return nnz;
    memcpy(row_ptr, rp, sizeof(int64_t) * (size_t)(n + 1));
    if (nnz <= cap) memcpy(col, c, sizeof(int32_t) * (size_t)nnz);
    free(rp);
    free(c);
    return nnz;
}

/* Cross query with cells: rows over A, columns into B.  Built on the joint
 * set (A then B) and filtered to the A-to-B pairs. */
int64_t or_xnbr_cells_alloc(const or_domain* d, int64_t na, const double* xa,
                            const double* ya, const double* ha, int64_t nb,
                            const double* xb, const double* yb, const double* hb,
                            int64_t** row_ptr_out, int32_t** col_out)
{
    int64_t n = na + nb;
    double* x = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* y = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* h = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    memcpy(x, xa, sizeof(double) * (size_t)na); memcpy(x + na, xb, sizeof(double) * (size_t)nb);
    memcpy(y, ya, sizeof(double) * (size_t)na); memcpy(y + na, yb, sizeof(double) * (size_t)nb);
    memcpy(h, ha, sizeof(double) * (size_t)na); memcpy(h + na, hb, sizeof(double) * (size_t)nb);
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, x, y, h, &rp, &col);
    free(x); free(y); free(h);
    if (nnz < 0) return nnz;
    int64_t* orp = (int64_t*)calloc((size_t)na + 1, sizeof(int64_t));
    int64_t cnt = 0;
    for (int64_t i = 0; i < na; ++i) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) if (col[k] >= na) ++cnt;
        orp[i + 1] = cnt;
    }
    int32_t* ocol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt > 0 ? cnt : 1));
    int64_t t = 0;
    for (int64_t i = 0; i < na; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] >= na) ocol[t++] = (int32_t)(col[k] - na);
    free(rp);
    free(col);
    *row_ptr_out = orp;
    *col_out = ocol;
    return cnt;
}

void or_free(void* p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Pass A: summation density (eq. sd-gather), variable-h correction beta     */
/* (eq. beta, d = 2), neighbour count and average pressure (eq. pavg), and   */
/* the limited Lind shifting displacement (eqs. shift-deltar, shift-limit).  */
/* ------------------------------------------------------------------------ */

/* Limited shifting displacement of particle i over its row (eqs.
 * shift-deltar and shift-limit).  READING: the garbled denominator
 * W(dx, xi h_ij) is the kernel at distance xi*h_ij with smoothing length
 * h_ij, so the ratio is f(r/h_ij) / f(xi); the gradient is at h_ij. */
static void shift_one(const or_domain* d, double rho0, int64_t i, const double* x,
                      const double* y, const double* h, const double* m,
                      const int64_t* rp, const int32_t* col, double* dxs, double* dys)
{
    double fxi = or_kf(OR_XI);
    double sx = 0.0, sy = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        int64_t j = col[k];
        double dx = mi_axis(d, 0, x[i] - x[j]);
        double dy = mi_axis(d, 1, y[i] - y[j]);
        double r = sqrt(dx * dx + dy * dy);
        if (r <= 0.0) continue;
        double hij = 0.5 * (h[i] + h[j]);
        double wr = or_kf(r / hij) / fxi;
        double coef = (m[j] / rho0) * (1.0 + 0.24 * ((wr * wr) * (wr * wr)));
        double t = coef * (or_dwdr(r, hij) / r);
        sx = sx + t * dx;
        sy = sy + t * dy;
    }
    double pref = -0.5 * (h[i] * h[i]);
    double ddx = pref * sx, ddy = pref * sy;
    double mag = sqrt(ddx * ddx + ddy * ddy);
    double lim = 0.25 * h[i];
    if (mag > lim) {
        double th = lim / mag;
        ddx = ddx * th;
        ddy = ddy * th;
    }
    *dxs = ddx;
    *dys = ddy;
}

/* READING: the average pressure of eq. (pavg) is formed as
 * p_i + (1/N_i) sum_j (p_j - p_i), the same mean written about p_i, so that a
 * uniform pressure gives p_avg = p exactly and the reduced pressure of eq.
 * (mom:pre) removes it exactly (a plain sum of N copies of a non-dyadic p
 * rounds, which would leave a force of rounding size on fluid at rest). */
void or_pass_a(const or_domain* d, const or_params* P, int64_t n, const double* x,
               const double* y, const double* h, const double* m, const double* p,
               const int64_t* rp, const int32_t* col, double* rho, double* beta,
               double* nnb, double* pavg, double* dxs, double* dys)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double sr = 0.0, sb = 0.0, sp = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            double dx = mi_axis(d, 0, x[i] - x[j]);
            double dy = mi_axis(d, 1, y[i] - y[j]);
            double r = sqrt(dx * dx + dy * dy);
            sr += m[j] * or_w(r, h[i]);
            sb += m[j] * r * or_dwdr(r, h[i]);
            sp += p[j] - p[i];
        }
        double N = (double)(rp[i + 1] - rp[i]);
        rho[i] = sr;
        beta[i] = -sb / (2.0 * sr);
        nnb[i] = N;
        pavg[i] = p[i] + sp / N;
        shift_one(d, P->rho0, i, x, y, h, m, rp, col, &dxs[i], &dys[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Pass B: EDAC pressure rate (eq. edac:sph) and momentum (eq. mom-sph).     */
/* READINGS: the diffusion term of eq. (edac:sph) is divided by              */
/* (r_ij^2 + eta_i) as the viscous term is; A_i, A_j and the third line of   */
/* eq. (mom-sph) are not used (remark after eq. mom-corr); eta_i =           */
/* 0.001 h_i^2; P_i from eq. (mom:pre) with p_avg from eq. (pavg).           */
/* READING (degenerate case the paper leaves open): beta_i <= 0 happens only */
/* when no neighbour lies inside particle i's own support; then P_i = 0 and  */
/* the sums scaled by 1/beta_i are dropped, so its rates stay finite.        */
/* ------------------------------------------------------------------------ */

/* ug, vg: the velocity used in the viscous term.  For fluid particles it is
 * u, v; for wall particles it is the no-slip ghost velocity of eq. (bc-wall)
 * (section 2.2).  NULL means ug = u, vg = v. */
void or_pass_b(const or_domain* d, const or_params* P, int64_t n, const double* x,
               const double* y, const double* u, const double* v, const double* p,
               const double* h, const double* m, const double* rho,
               const double* beta, const double* pavg, const double* dxs,
               const double* dys, double dt, const int64_t* rp, const int32_t* col,
               const double* ug, const double* vg,
               double* dpdt, double* dudt, double* dvdt)
{
    const double rho0 = P->rho0, cs = P->cs, nu = P->nu, ae = P->alpha_e;
    if (!ug) ug = u;
    if (!vg) vg = v;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double Pi = beta[i] > 0.0 ? (p[i] - pavg[i]) / (rho[i] * rho[i] * beta[i]) : 0.0;
        double nui = ae * cs * h[i] / 8.0;
        double eta = 0.001 * h[i] * h[i];
        double s_div = 0.0, s_dif = 0.0, gx = 0.0, gy = 0.0, vx = 0.0, vy = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            double dx = mi_axis(d, 0, x[i] - x[j]);
            double dy = mi_axis(d, 1, y[i] - y[j]);
            double r2 = dx * dx + dy * dy;
            double r = sqrt(r2);
            double gix = 0.0, giy = 0.0, gjx = 0.0, gjy = 0.0;
            if (r > 0.0) {
                double fi = or_dwdr(r, h[i]) / r;
                double fj = or_dwdr(r, h[j]) / r;
                gix = fi * dx; giy = fi * dy;
                gjx = fj * dx; gjy = fj * dy;
            }
            double gbx = 0.5 * (gix + gjx), gby = 0.5 * (giy + gjy);
            double uij = u[i] - u[j], vij = v[i] - v[j];
            double Vj = m[j] / rho[j];
            double Pj = beta[j] <= 0.0 ? 0.0
                      : P->pref_mode ? (p[j] - pavg[i]) / (rho[j] * rho[j] * beta[j])
                                     : (p[j] - pavg[j]) / (rho[j] * rho[j] * beta[j]);
            double nuj = ae * cs * h[j] / 8.0;
            double nuij = 4.0 * nui * nuj / (nui + nuj);
            double rdotg = dx * gbx + dy * gby;
            /* divergence: sum V_j u_ij . gradW(h_i) */
            s_div += Vj * (uij * gix + vij * giy);
            /* pressure diffusion */
            s_dif += Vj * nuij * (p[i] - p[j]) * rdotg / (r2 + eta);
            /* pressure gradient G_i = sum m_j (P_i gradW_i + P_j gradW_j) */
            gx += m[j] * (Pi * gix + Pj * gjx);
            gy += m[j] * (Pi * giy + Pj * gjy);
            /* viscous */
            double cvis = m[j] * (4.0 * nu / (rho[i] + rho[j])) * rdotg / (r2 + eta);
            vx += cvis * (ug[i] - ug[j]);
            vy += cvis * (vg[i] - vg[j]);
        }
        double b = beta[i];
        double edac = b > 0.0 ? (rho0 * cs * cs / b) * s_div + s_dif / b : 0.0;
        dpdt[i] = edac + (dxs[i] / dt) * gx + (dys[i] / dt) * gy;
        dudt[i] = -gx + (b > 0.0 ? vx / b : 0.0) + P->fx;
        dvdt[i] = -gy + (b > 0.0 ? vy / b : 0.0) + P->fy;
    }
}

/* Per-particle scales of the rates for condition-aware comparisons: for
 * every field, the sum over j of the magnitudes of its pair terms, as
 * pass A and pass B above form them (the size of the quantity a rounding
 * error in those terms is relative to).  Fields, n entries each, in this
 * order: rho, beta, pavg, dxs, dys, dpdt, dudt, dvdt.
 *   rho:  sum |m_j W(r_ij, h_i)|;
 *   beta: sum |m_j r_ij dW/dr(r_ij, h_i)| / (2 rho_i);
 *   pavg: |p_i| + sum |p_j - p_i| / N_i (the terms of p_i + mean(p_j - p_i));
 *   dxs, dys: theta (h_i^2 / 2) sum |t_j| (|dx_j| + |dy_j|), t_j the scalar
 *         factor of the shifting sum of eq. (shift-deltar) and theta the
 *         limiter of eq. (shift-limit) (both components, because the limiter
 *         couples them);
 *   dpdt: (rho0 c^2 / |beta_i|) sum V_j (|u_ij gradW_i,x| + |v_ij gradW_i,y|)
 *         + sum V_j |nu_ij (p_i - p_j) r_ij . gradW_ij| / ((r_ij^2 + eta_i) |beta_i|)
 *         + (|dxs_i| S_x + |dys_i| S_y) / dt + (s_dxs |G_x| + s_dys |G_y|) / dt,
 *         S_x = sum m_j (|P_i| |gradW_i,x| + |P_j| |gradW_j,x|) with the
 *         reduced pressures of eq. (mom:pre) taken at the size of what they
 *         are formed from, |P_i| = (|p_i| + |p_avg,i|) / (rho_i^2 |beta_i|)
 *         and |P_j| = (|p_j| + |p_avg|) / (rho_j^2 |beta_j|) (p - p_avg
 *         cancels where the pressure is nearly uniform about an offset, and
 *         a rounding of p_avg at that offset is then all of it), G the signed
 *         pressure-gradient sum and s_dxs, s_dys the shift scales (the error
 *         of the shift enters through the transport-velocity term);
 *   dudt: S_x + sum |c_ij (ug_i - ug_j)| / |beta_i| + |f_x|, c_ij the
 *         viscous factor of eq. (mom-sph); dvdt likewise.
 * Sums scaled by 1/beta_i are dropped where beta_i <= 0, as in pass B.
 * kind (may be NULL: all fluid): the boundary pass computes u, v, p and the
 * ghost velocity of non-fluid particles from Shepard averages, which carry
 * their own rounding, so a difference a_i - a_j of those values over a pair
 * with a non-fluid member is taken at mag_i + mag_j, mag being the size of
 * what each value is formed from: mag (5 n doubles: p, u, v, ug, vg) as
 * or_boundary_mags writes it, or |a| where mag is NULL. */
void or_rate_scales(const or_domain* d, const or_params* P, int64_t n, const double* x,
                    const double* y, const double* u, const double* v, const double* p,
                    const double* h, const double* m, const double* rho,
                    const double* beta, const double* pavg, const double* dxs,
                    const double* dys, double dt, const int64_t* rp, const int32_t* col,
                    const double* ug, const double* vg, const int32_t* kind,
                    const double* mag, double* sc)
{
    const double rho0 = P->rho0, cs = P->cs, nu = P->nu, ae = P->alpha_e;
    if (!ug) ug = u;
    if (!vg) vg = v;
    const double fxi = or_kf(OR_XI);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double s_rho = 0.0, s_beta = 0.0, s_p = 0.0, s_sh = 0.0, sx = 0.0, sy = 0.0;
        double s_div = 0.0, s_dif = 0.0, Sx = 0.0, Sy = 0.0, Gx = 0.0, Gy = 0.0;
        double s_vx = 0.0, s_vy = 0.0;
        double Pi = beta[i] > 0.0 ? (p[i] - pavg[i]) / (rho[i] * rho[i] * beta[i]) : 0.0;
        const double pmi = mag ? mag[i] : fabs(p[i]);
        double Pai = beta[i] > 0.0 ? (pmi + fabs(pavg[i])) / (rho[i] * rho[i] * beta[i]) : 0.0;
        double nui = ae * cs * h[i] / 8.0;
        double eta = 0.001 * h[i] * h[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            double dx = mi_axis(d, 0, x[i] - x[j]);
            double dy = mi_axis(d, 1, y[i] - y[j]);
            double r2 = dx * dx + dy * dy;
            double r = sqrt(r2);
            /* |a_i - a_j|, or |a_i| + |a_j| over a pair with a boundary member */
            const int bnd = kind && (kind[i] != 0 || kind[j] != 0);
#define OR_MAG(a, f, q) (mag ? mag[(f) * n + (q)] : fabs((a)[q]))
#define OR_DABS_F(a, f) (bnd ? OR_MAG(a, f, i) + OR_MAG(a, f, j) : fabs((a)[i] - (a)[j]))
            s_rho += fabs(m[j] * or_w(r, h[i]));
            s_beta += fabs(m[j] * r * or_dwdr(r, h[i]));
            s_p += OR_DABS_F(p, 0);
            double gix = 0.0, giy = 0.0, gjx = 0.0, gjy = 0.0;
            if (r > 0.0) {
                double hij = 0.5 * (h[i] + h[j]);
                double wr = or_kf(r / hij) / fxi;
                double t = (m[j] / rho0) * (1.0 + 0.24 * ((wr * wr) * (wr * wr))) *
                           (or_dwdr(r, hij) / r);
                sx += t * dx;
                sy += t * dy;
                s_sh += fabs(t) * (fabs(dx) + fabs(dy));
                double fi = or_dwdr(r, h[i]) / r;
                double fj = or_dwdr(r, h[j]) / r;
                gix = fi * dx; giy = fi * dy;
                gjx = fj * dx; gjy = fj * dy;
            }
            double gbx = 0.5 * (gix + gjx), gby = 0.5 * (giy + gjy);
            double Vj = m[j] / rho[j];
            double pref_j = P->pref_mode ? pavg[i] : pavg[j];
            double Pj = beta[j] <= 0.0 ? 0.0 : (p[j] - pref_j) / (rho[j] * rho[j] * beta[j]);
            double Paj = beta[j] <= 0.0 ? 0.0
                       : ((mag ? mag[j] : fabs(p[j])) + fabs(pref_j)) / (rho[j] * rho[j] * beta[j]);
            double nuj = ae * cs * h[j] / 8.0;
            double nuij = 4.0 * nui * nuj / (nui + nuj);
            double rdotg = dx * gbx + dy * gby;
            s_div += Vj * (OR_DABS_F(u, 1) * fabs(gix) + OR_DABS_F(v, 2) * fabs(giy));
            s_dif += Vj * fabs(nuij * rdotg) * OR_DABS_F(p, 0) / (r2 + eta);
            Sx += m[j] * (Pai * fabs(gix) + Paj * fabs(gjx));
            Sy += m[j] * (Pai * fabs(giy) + Paj * fabs(gjy));
            Gx += m[j] * (Pi * gix + Pj * gjx);
            Gy += m[j] * (Pi * giy + Pj * gjy);
            double cvis = m[j] * (4.0 * nu / (rho[i] + rho[j])) * rdotg / (r2 + eta);
            s_vx += fabs(cvis) * OR_DABS_F(ug, 3);
            s_vy += fabs(cvis) * OR_DABS_F(vg, 4);
        }
        double N = (double)(rp[i + 1] - rp[i]);
        double pref = 0.5 * (h[i] * h[i]);
        double mag = pref * sqrt(sx * sx + sy * sy);
        double lim = 0.25 * h[i];
        double th = mag > lim ? lim / mag : 1.0;
        double s_shift = th * pref * s_sh;
        double b = beta[i];
        double ib = b > 0.0 ? 1.0 / b : 0.0;
        sc[0 * n + i] = s_rho;
        sc[1 * n + i] = s_beta / (2.0 * fabs(rho[i]));
        sc[2 * n + i] = pmi + (N > 0 ? s_p / N : 0.0);
#undef OR_MAG
#undef OR_DABS_F
        sc[3 * n + i] = s_shift;
        sc[4 * n + i] = s_shift;
        sc[5 * n + i] = rho0 * cs * cs * ib * s_div + s_dif * ib +
                        (fabs(dxs[i]) * Sx + fabs(dys[i]) * Sy) / dt +
                        s_shift * (fabs(Gx) + fabs(Gy)) / dt;
        sc[6 * n + i] = Sx + s_vx * ib + fabs(P->fx);
        sc[7 * n + i] = Sy + s_vy * ib + fabs(P->fy);
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary particles, section 2.2.  Kinds: 0 fluid, 1 solid (dummy wall     */
/* particles of Adami et al.), 2 inlet, 3 outlet.  For every non-fluid       */
/* particle b the Shepard sums of eq. (shepard) run over its fluid           */
/* neighbours f with W(r_bf, h_bf), h_bf = (h_b + h_f)/2:                    */
/*   solid:  p_b by eq. (bc-pre) with g the body force and a_w the wall      */
/*           acceleration; ghost velocity 2 u_b - u^_b (eq. bc-wall), used    */
/*           in the viscous term; u_b (the prescribed wall velocity) stays   */
/*           and is the one the pressure equation sees (no penetration);     */
/*   inlet and outlet, io_mode 0: the inlet keeps its prescribed velocity    */
/*     and takes p_b = Shepard average of the fluid pressure; the outlet     */
/*     takes u_b, v_b, p_b = Shepard averages of the fluid values (a zero-   */
/*     gradient extrapolation);                                              */
/*   inlet and outlet, io_mode 1 (the non-reflecting condition of Lastiwka   */
/*     et al. that the paper uses): the characteristic variables of the      */
/*     Euler equations linearised about the reference state (u_r, v_r, p_r,  */
/*     rho0) along the flow direction +x,                                    */
/*       J2 = rho0 c (u - u_r) + (p - p_r)   (carried with u + c),           */
/*       J3 = -rho0 c (u - u_r) + (p - p_r)  (carried with u - c),           */
/*     are Shepard-averaged from the fluid where they leave the domain and   */
/*     set to 0 where they enter it: at the (upstream) inlet J2 = 0 and J3   */
/*     is extrapolated, v = v_r; at the (downstream) outlet J3 = 0 and J2    */
/*     is extrapolated, v is extrapolated.  Then p = p_r + (J2 + J3)/2 and   */
/*     u = u_r + (J2 - J3)/(2 rho0 c).  The Shepard average is linear, so    */
/*     the extrapolated J is that of the averaged u and p.  READING: the     */
/*     entropy variable J1 = -c^2 (rho - rho0) + (p - p_r) only fixes the    */
/*     density, which the summation density supplies, so it is not used.    */
/* READING: rho_f in eq. (bc-pre) is the stored density (the one from the    */
/* latest summation).  A particle with no fluid neighbour keeps u, v, p and  */
/* its ghost velocity is u; by the symmetry of N no fluid particle sees it.  */
/* ------------------------------------------------------------------------ */

enum { OR_FLUID = 0, OR_SOLID = 1, OR_INLET = 2, OR_OUTLET = 3 };

typedef struct {
    double awx, awy;   /* wall acceleration a_w of eq. (bc-pre) */
    int32_t io_mode;   /* inlet/outlet rule: 0 zero-gradient, 1 characteristic */
    double ur, vr, pr; /* reference (prescribed inlet) state of io_mode 1 */
} or_bc;

void or_boundary(const or_domain* d, const or_params* P, const or_bc* B, int64_t n,
                 const double* x, const double* y, const double* h, const double* rho,
                 const int32_t* kind, const int64_t* rp, const int32_t* col, double* u,
                 double* v, double* p, double* ug, double* vg)
{
    for (int64_t i = 0; i < n; ++i) {
        ug[i] = u[i];
        vg[i] = v[i];
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        if (kind[b] == OR_FLUID) continue;
        double S = 0.0, su = 0.0, sv = 0.0, sp = 0.0, srx = 0.0, sry = 0.0;
        for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
            int64_t f = col[k];
            if (kind[f] != OR_FLUID) continue;
            double dx = mi_axis(d, 0, x[b] - x[f]);
            double dy = mi_axis(d, 1, y[b] - y[f]);
            double r = sqrt(dx * dx + dy * dy);
            double w = or_w(r, 0.5 * (h[b] + h[f]));
            S += w;
            su += u[f] * w;
            sv += v[f] * w;
            sp += p[f] * w;
            srx += rho[f] * dx * w;
            sry += rho[f] * dy * w;
        }
        if (!(S > 0.0)) continue;
        if (kind[b] == OR_SOLID) {
            p[b] = (sp + ((P->fx - B->awx) * srx + (P->fy - B->awy) * sry)) / S;
            ug[b] = 2.0 * u[b] - su / S;
            vg[b] = 2.0 * v[b] - sv / S;
        } else if (B->io_mode == 1) {
            double zc = P->rho0 * P->cs;
            double du = su / S - B->ur;
            double dp = sp / S - B->pr;
            if (kind[b] == OR_INLET) {
                double j3 = dp - zc * du;
                u[b] = B->ur - j3 / (2.0 * zc);
                v[b] = B->vr;
                p[b] = B->pr + 0.5 * j3;
            } else {
                double j2 = dp + zc * du;
                u[b] = B->ur + j2 / (2.0 * zc);
                v[b] = sv / S;
                p[b] = B->pr + 0.5 * j2;
            }
            ug[b] = u[b];
            vg[b] = v[b];
        } else if (kind[b] == OR_INLET) {
            p[b] = sp / S;
        } else {
            u[b] = su / S;
            v[b] = sv / S;
            p[b] = sp / S;
            ug[b] = u[b];
            vg[b] = v[b];
        }
    }
}

/* One full rate evaluation: neighbours (cell list), the boundary pass when
 * kind is given (it overwrites p, and u, v of outlet particles, in place;
 * rho_in is the stored density it uses), pass A, pass B. */
/* Sizes of the values the boundary pass forms (for or_rate_scales): for
 * every particle, mag[f n + i] with f = 0..4 for p, u, v, ug, vg.  Fluid
 * particles and boundary particles without fluid neighbours: |value|.
 * Boundary particles: the same Shepard sums as or_boundary with every term
 * taken in magnitude, e.g. for a solid (sum |p_f| w + |g_x| sum |rho_f dx| w
 * + |g_y| sum |rho_f dy| w) / S for p and 2 |u_b| + sum |u_f| w / S for its
 * ghost velocity; for the characteristic rule, |p_r| + |J|_mag / 2 and
 * |u_r| + |J|_mag / (2 rho0 c) with |J|_mag = sum |p_f| w / S + |p_r| +
 * rho0 c (sum |u_f| w / S + |u_r|).  u, v, p, ug, vg: the values after the
 * boundary pass. */
static void or_boundary_mags(const or_domain* d, const or_params* P, const or_bc* B, int64_t n,
                             const double* x, const double* y, const double* h,
                             const double* rho, const int32_t* kind, const int64_t* rp,
                             const int32_t* col, const double* u0, const double* v0,
                             const double* u, const double* v, const double* p,
                             const double* ug, const double* vg, double* mag)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        mag[0 * n + b] = fabs(p[b]);
        mag[1 * n + b] = fabs(u[b]);
        mag[2 * n + b] = fabs(v[b]);
        mag[3 * n + b] = fabs(ug[b]);
        mag[4 * n + b] = fabs(vg[b]);
        if (kind[b] == OR_FLUID) continue;
        double S = 0.0, su = 0.0, sv = 0.0, sp = 0.0, srx = 0.0, sry = 0.0;
        for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
            int64_t f = col[k];
            if (kind[f] != OR_FLUID) continue;
            double dx = mi_axis(d, 0, x[b] - x[f]);
            double dy = mi_axis(d, 1, y[b] - y[f]);
            double r = sqrt(dx * dx + dy * dy);
            double w = or_w(r, 0.5 * (h[b] + h[f]));
            S += w;
            su += fabs(u[f]) * w;
            sv += fabs(v[f]) * w;
            sp += fabs(p[f]) * w;
            srx += fabs(rho[f] * dx) * w;
            sry += fabs(rho[f] * dy) * w;
        }
        if (!(S > 0.0)) continue;
        if (kind[b] == OR_SOLID) {
            mag[0 * n + b] = (sp + fabs(P->fx - B->awx) * srx + fabs(P->fy - B->awy) * sry) / S;
            mag[3 * n + b] = 2.0 * fabs(u0[b]) + su / S;
            mag[4 * n + b] = 2.0 * fabs(v0[b]) + sv / S;
        } else if (B->io_mode == 1) {
            double zc = P->rho0 * P->cs;
            double jm = sp / S + fabs(B->pr) + zc * (su / S + fabs(B->ur));
            mag[0 * n + b] = fabs(B->pr) + 0.5 * jm;
            mag[1 * n + b] = fabs(B->ur) + jm / (2.0 * zc);
            mag[2 * n + b] = kind[b] == OR_INLET ? fabs(B->vr) : sv / S;
            mag[3 * n + b] = mag[1 * n + b];
            mag[4 * n + b] = mag[2 * n + b];
        } else if (kind[b] == OR_INLET) {
            mag[0 * n + b] = sp / S;
        } else {
            mag[0 * n + b] = sp / S;
            mag[1 * n + b] = su / S;
            mag[2 * n + b] = sv / S;
            mag[3 * n + b] = su / S;
            mag[4 * n + b] = sv / S;
        }
    }
}

/* The same, also writing the per-particle scales of or_rate_scales (8 n
 * doubles) when sc is not NULL. */
int or_rates_k_scaled(const or_domain* d, const or_params* P, const or_bc* B, int64_t n,
                      const double* x, const double* y, double* u, double* v, double* p,
                      const double* h, const double* m, const int32_t* kind,
                      const double* rho_in, double dt, double* rho, double* beta, double* nnb,
                      double* pavg, double* dxs, double* dys, double* dpdt, double* dudt,
                      double* dvdt, double* sc)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, x, y, h, &rp, &col);
    if (nnz < 0) return (int)nnz;
    double *ug = NULL, *vg = NULL, *mag = NULL, *u0 = NULL, *v0 = NULL;
    if (kind) {
        size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
        ug = malloc(sz);
        vg = malloc(sz);
        if (sc) {
            mag = malloc(5 * sz);
            u0 = malloc(sz);
            v0 = malloc(sz);
        }
        if (!ug || !vg || (sc && (!mag || !u0 || !v0))) {
            free(ug); free(vg); free(mag); free(u0); free(v0); free(rp); free(col);
            return OR_E_NOMEM;
        }
        if (sc) {
            memcpy(u0, u, sizeof(double) * (size_t)n);
            memcpy(v0, v, sizeof(double) * (size_t)n);
        }
        or_boundary(d, P, B, n, x, y, h, rho_in, kind, rp, col, u, v, p, ug, vg);
        if (sc)
            or_boundary_mags(d, P, B, n, x, y, h, rho_in, kind, rp, col, u0, v0, u, v, p, ug,
                             vg, mag);
    }
    or_pass_a(d, P, n, x, y, h, m, p, rp, col, rho, beta, nnb, pavg, dxs, dys);
    or_pass_b(d, P, n, x, y, u, v, p, h, m, rho, beta, pavg, dxs, dys, dt, rp, col, ug, vg,
              dpdt, dudt, dvdt);
    if (sc)
        or_rate_scales(d, P, n, x, y, u, v, p, h, m, rho, beta, pavg, dxs, dys, dt, rp, col, ug,
                       vg, kind, mag, sc);
    free(ug);
    free(vg);
    free(mag);
    free(u0);
    free(v0);
    free(rp);
    free(col);
    return OR_OK;
}

int or_rates_k(const or_domain* d, const or_params* P, const or_bc* B, int64_t n,
               const double* x, const double* y, double* u, double* v, double* p,
               const double* h, const double* m, const int32_t* kind, const double* rho_in,
               double dt, double* rho, double* beta, double* nnb, double* pavg, double* dxs,
               double* dys, double* dpdt, double* dudt, double* dvdt)
{
    return or_rates_k_scaled(d, P, B, n, x, y, u, v, p, h, m, kind, rho_in, dt, rho, beta, nnb,
                             pavg, dxs, dys, dpdt, dudt, dvdt, NULL);
}

/* ------------------------------------------------------------------------ */
/* Force on the solid (dummy wall) particles, section 2.3, eq. (force-sph):  */
/* for every solid particle i, over its fluid neighbours j,                  */
/*   f_p,i    = -m_i sum_j m_j (P_i gradW(r_ij, h_i) + P_j gradW(r_ij, h_j))  */
/*   f_visc,i =  m_i (1/beta_i) sum_j m_j 4 nu/(rho_i + rho_j)              */
/*                 (r_ij . gradW_ij)/(r_ij^2 + eta_i) u_ij                   */
/* and the totals over all solid particles.  eta_i, beta_i and u_ij (with    */
/* the ghost velocity of the solid particle) are those of the momentum       */
/* equation in pass B above.                                                  */
/* READING: P_i = p_i/(rho_i^2 beta_i), P_j = p_j/(rho_j^2 beta_j), without  */
/* the pressure reduction of eq. (mom:pre).  The reduction removes the local */
/* mean pressure, which has no net effect inside the fluid; over the one-    */
/* sided sums at a body surface it removes the pressure the force integrates */
/* (with it, a body in a linear pressure field feels a force that vanishes   */
/* like h instead of -grad p times its area).                                 */
/* READING: gradW_ij, the kernel gradient at h_ij in the viscous sum, is the  */
/* average of the gradients at h_i and h_j (eq. dw-avg), as in the momentum  */
/* equation, so the force is m_i times the fluid part of the solid           */
/* particle's own momentum sums.                                              */
/* One evaluation's state is formed first as in or_rates_k: neighbours, the  */
/* boundary pass (on u, v, p in place), pass A.                               */
/* out[0..3] = f_p,x, f_p,y, f_visc,x, f_visc,y; out[4..7] = the sums of the  */
/* absolute values of the pair terms of each (for rounding bounds).          */
/* ------------------------------------------------------------------------ */
int or_body_force(const or_domain* d, const or_params* P, const or_bc* B, int64_t n,
                  const double* x, const double* y, double* u, double* v, double* p,
                  const double* h, const double* m, const int32_t* kind, const double* rho_in,
                  double* out)
{
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, x, y, h, &rp, &col);
    if (nnz < 0) return (int)nnz;
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double* buf = malloc(sz * 8);
    if (!buf) {
        free(rp); free(col);
        return OR_E_NOMEM;
    }
    double *ug = buf, *vg = buf + n, *rho = buf + 2 * n, *beta = buf + 3 * n, *nnb = buf + 4 * n,
           *pavg = buf + 5 * n, *dxs = buf + 6 * n, *dys = buf + 7 * n;
    or_boundary(d, P, B, n, x, y, h, rho_in, kind, rp, col, u, v, p, ug, vg);
    or_pass_a(d, P, n, x, y, h, m, p, rp, col, rho, beta, nnb, pavg, dxs, dys);
    const double nu = P->nu;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != OR_SOLID) continue;
        const double Pi = beta[i] > 0.0 ? p[i] / (rho[i] * rho[i] * beta[i]) : 0.0;
        const double eta = 0.001 * h[i] * h[i];
        double fpx = 0.0, fpy = 0.0, fvx = 0.0, fvy = 0.0;
        double apx = 0.0, apy = 0.0, avx = 0.0, avy = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = col[k];
            if (kind[j] != OR_FLUID) continue;
            const double dx = mi_axis(d, 0, x[i] - x[j]);
            const double dy = mi_axis(d, 1, y[i] - y[j]);
            const double r2 = dx * dx + dy * dy;
            const double r = sqrt(r2);
            double gix = 0.0, giy = 0.0, gjx = 0.0, gjy = 0.0;
            if (r > 0.0) {
                const double fi = or_dwdr(r, h[i]) / r;
                const double fj = or_dwdr(r, h[j]) / r;
                gix = fi * dx; giy = fi * dy;
                gjx = fj * dx; gjy = fj * dy;
            }
            const double Pj = beta[j] <= 0.0 ? 0.0 : p[j] / (rho[j] * rho[j] * beta[j]);
            const double tpx = -m[i] * m[j] * (Pi * gix + Pj * gjx);
            const double tpy = -m[i] * m[j] * (Pi * giy + Pj * gjy);
            fpx += tpx; fpy += tpy;
            apx += fabs(tpx); apy += fabs(tpy);
            if (beta[i] > 0.0) {
                const double rdotg = dx * 0.5 * (gix + gjx) + dy * 0.5 * (giy + gjy);
                const double cvis = m[j] * (4.0 * nu / (rho[i] + rho[j])) * rdotg / (r2 + eta);
                const double tvx = m[i] * cvis * (ug[i] - ug[j]) / beta[i];
                const double tvy = m[i] * cvis * (vg[i] - vg[j]) / beta[i];
                fvx += tvx; fvy += tvy;
                avx += fabs(tvx); avy += fabs(tvy);
            }
        }
        out[0] += fpx; out[1] += fpy; out[2] += fvx; out[3] += fvy;
        out[4] += apx; out[5] += apy; out[6] += avx; out[7] += avy;
    }
    free(buf);
    free(rp);
    free(col);
    return OR_OK;
}

int or_rates(const or_domain* d, const or_params* P, int64_t n, const double* x,
             const double* y, const double* u, const double* v, const double* p,
             const double* h, const double* m, double dt, double* rho, double* beta,
             double* nnb, double* pavg, double* dxs, double* dys, double* dpdt,
             double* dudt, double* dvdt)
{
    return or_rates_k(d, P, NULL, n, x, y, (double*)u, (double*)v, (double*)p, h, m, NULL, NULL,
                      dt, rho, beta, nnb, pavg, dxs, dys, dpdt, dudt, dvdt);
}

/* ------------------------------------------------------------------------ */
/* Predict-evaluate-correct integrator, eqs. (int-pre) and (int-cor), with   */
/* the transport velocity u~ = u + dr/dt of eq. (shift-tvf).  Neighbours are */
/* rebuilt before each of the two evaluations per step.  Positions on        */
/* periodic axes are wrapped into [lo, hi).                                  */
/* With kinds: fluid particles are integrated as above; solid particles stay */
/* in place; inlet and outlet particles move with their own velocity (no     */
/* shifting), the half step with u^n, the full step with the velocity of the */
/* half-step boundary pass.  Every non-fluid particle keeps the half-step    */
/* boundary values of u, v, p at the end of the step.  rho carries the       */
/* stored density in and the latest summation density out.                 */
/* ------------------------------------------------------------------------ */

int or_step_k(const or_domain* d, const or_params* P, const or_bc* B, int64_t n, double* x,
              double* y, double* u, double* v, double* p, double* h, const double* m,
              const int32_t* kind, double* rho, double dt, int64_t nsteps)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *rn = malloc(sz), *beta = malloc(sz), *nnb = malloc(sz), *pavg = malloc(sz);
    double *dxs = malloc(sz), *dys = malloc(sz), *ap = malloc(sz), *au = malloc(sz), *av = malloc(sz);
    double *xh = malloc(sz), *yh = malloc(sz), *uh = malloc(sz), *vh = malloc(sz), *ph = malloc(sz);
    int rc = OR_OK;
    if (!rn || !beta || !nnb || !pavg || !dxs || !dys || !ap || !au || !av || !xh || !yh || !uh ||
        !vh || !ph)
        rc = OR_E_NOMEM;
    for (int64_t s = 0; s < nsteps && rc == OR_OK; ++s) {
        rc = or_rates_k(d, P, B, n, x, y, u, v, p, h, m, kind, rho, dt, rn, beta, nnb, pavg, dxs,
                        dys, ap, au, av);
        if (rc) break;
        memcpy(rho, rn, sz);
        for (int64_t i = 0; i < n; ++i) {
            int k = kind ? kind[i] : OR_FLUID;
            if (k != OR_FLUID) {
                double adv = (k == OR_INLET || k == OR_OUTLET) ? 1.0 : 0.0;
                xh[i] = adv > 0.0 ? wrap_axis(d, 0, x[i] + 0.5 * dt * u[i]) : x[i];
                yh[i] = adv > 0.0 ? wrap_axis(d, 1, y[i] + 0.5 * dt * v[i]) : y[i];
                uh[i] = u[i];
                vh[i] = v[i];
                ph[i] = p[i];
                continue;
            }
            uh[i] = u[i] + 0.5 * dt * au[i];
            vh[i] = v[i] + 0.5 * dt * av[i];
            double tu = uh[i] + dxs[i] / dt;
            double tv = vh[i] + dys[i] / dt;
            xh[i] = wrap_axis(d, 0, x[i] + 0.5 * dt * tu);
            yh[i] = wrap_axis(d, 1, y[i] + 0.5 * dt * tv);
            ph[i] = p[i] + 0.5 * dt * ap[i];
        }
        rc = or_rates_k(d, P, B, n, xh, yh, uh, vh, ph, h, m, kind, rho, dt, rn, beta, nnb, pavg,
                        dxs, dys, ap, au, av);
        if (rc) break;
        memcpy(rho, rn, sz);
        for (int64_t i = 0; i < n; ++i) {
            int k = kind ? kind[i] : OR_FLUID;
            if (k != OR_FLUID) {
                if (k == OR_INLET || k == OR_OUTLET) {
                    x[i] = wrap_axis(d, 0, x[i] + dt * uh[i]);
                    y[i] = wrap_axis(d, 1, y[i] + dt * vh[i]);
                }
                u[i] = uh[i];
                v[i] = vh[i];
                p[i] = ph[i];
                continue;
            }
            double un = u[i] + dt * au[i];
            double vn = v[i] + dt * av[i];
            double tu = un + dxs[i] / dt;
            double tv = vn + dys[i] / dt;
            x[i] = wrap_axis(d, 0, x[i] + dt * tu);
            y[i] = wrap_axis(d, 1, y[i] + dt * tv);
            u[i] = un;
            v[i] = vn;
            p[i] = p[i] + dt * ap[i];
        }
    }
    free(rn); free(beta); free(nnb); free(pavg); free(dxs); free(dys); free(ap); free(au); free(av);
    free(xh); free(yh); free(uh); free(vh); free(ph);
    return rc;
}

int or_step(const or_domain* d, const or_params* P, int64_t n, double* x, double* y,
            double* u, double* v, double* p, double* h, const double* m, double dt,
            int64_t nsteps, double* rho_out)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double* rho = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!rho) return OR_E_NOMEM;
    int rc = or_step_k(d, P, NULL, n, x, y, u, v, p, h, m, NULL, rho, dt, nsteps);
    if (rho_out && rc == OR_OK) memcpy(rho_out, rho, sz);
    free(rho);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* A body with prescribed rigid motion (the moving bodies of section 3.3):   */
/* every solid particle (kind 1) is translated by (dx, dy), wrapped on       */
/* periodic axes, and takes the body's velocity (vx, vy).  The wall          */
/* acceleration a_w of eq. (bc-pre) is the caller's (or_bc).                 */
/* ------------------------------------------------------------------------ */

void or_move_solids(const or_domain* d, int64_t n, const int32_t* kind, double dx, double dy,
                    double vx, double vy, double* x, double* y, double* u, double* v)
{
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != OR_SOLID) continue;
        x[i] = wrap_axis(d, 0, x[i] + dx);
        y[i] = wrap_axis(d, 1, y[i] + dy);
        u[i] = vx;
        v[i] = vy;
    }
}

/* Inlet and outlet (section 2.2): after a step, on the pre-update kinds,    */
/*   an inlet particle at x >= x_in becomes fluid and a copy of it (same y,  */
/*   h, mass, m_ref, u, v, p, rho) re-enters the inlet at x - len_in;        */
/*   a fluid particle at x >= x_out becomes an outlet particle;              */
/*   an outlet particle at x >= x_out + len_out is deleted.                  */
/* Deleted slots are removed by stable compaction and the inlet copies are   */
/* appended in ascending order of their source slot.  origin[new] is the     */
/* old slot (of the source, for a copy).  Returns the new count, or          */
/* OR_E_CAPACITY (state unchanged) when the result exceeds cap; counts[0..3] */
/* = appended, deleted, inlet->fluid, fluid->outlet.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    double x_in, len_in, x_out, len_out;
} or_io;

int64_t or_inout(const or_io* io, int64_t n, int64_t cap, double* x, double* y, double* u,
                 double* v, double* p, double* rho, double* h, double* mref, int64_t* mq,
                 int32_t* kind, int64_t* origin, int64_t* counts)
{
    int64_t na = 0, nd = 0, nf = 0, no = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] == OR_INLET && x[i] >= io->x_in) ++na;
        if (kind[i] == OR_OUTLET && x[i] >= io->x_out + io->len_out) ++nd;
    }
    for (int k = 0; k < 4; ++k) counts[k] = 0;
    if (n - nd + na > cap) return OR_E_CAPACITY;
    size_t m = (size_t)(n > 0 ? n : 1);
    int32_t* nk = malloc(m * sizeof(int32_t));
    int64_t* src = malloc((size_t)(n + na > 0 ? n + na : 1) * sizeof(int64_t));
    if (!nk || !src) { free(nk); free(src); return OR_E_NOMEM; }
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i) {
        nk[i] = kind[i];
        if (kind[i] == OR_INLET && x[i] >= io->x_in) { nk[i] = OR_FLUID; ++nf; }
        else if (kind[i] == OR_FLUID && x[i] >= io->x_out) { nk[i] = OR_OUTLET; ++no; }
        if (kind[i] == OR_OUTLET && x[i] >= io->x_out + io->len_out) continue;
        src[t++] = i;
    }
    int64_t nkeep = t;
    for (int64_t i = 0; i < n; ++i)
        if (kind[i] == OR_INLET && x[i] >= io->x_in) src[t++] = i;
    /* gather every array into the new order through a temporary */
    double* arrs[] = {x, y, u, v, p, rho, h, mref};
    double* tmpd = malloc((size_t)(t > 0 ? t : 1) * sizeof(double));
    int64_t* tmpq = malloc((size_t)(t > 0 ? t : 1) * sizeof(int64_t));
    int32_t* tmpk = malloc((size_t)(t > 0 ? t : 1) * sizeof(int32_t));
    if (!tmpd || !tmpq || !tmpk) {
        free(nk); free(src); free(tmpd); free(tmpq); free(tmpk);
        return OR_E_NOMEM;
    }
    for (int a = 0; a < 8; ++a) {
        double* A = arrs[a];
        for (int64_t k = 0; k < t; ++k) tmpd[k] = A[src[k]];
        if (a == 0)
            for (int64_t k = nkeep; k < t; ++k) tmpd[k] = A[src[k]] - io->len_in;
        memcpy(A, tmpd, (size_t)t * sizeof(double));
    }
    for (int64_t k = 0; k < t; ++k) tmpq[k] = mq[src[k]];
    memcpy(mq, tmpq, (size_t)t * sizeof(int64_t));
    for (int64_t k = 0; k < t; ++k) tmpk[k] = k < nkeep ? nk[src[k]] : OR_INLET;
    memcpy(kind, tmpk, (size_t)t * sizeof(int32_t));
    for (int64_t k = 0; k < t; ++k) origin[k] = src[k];
    counts[0] = na; counts[1] = nd; counts[2] = nf; counts[3] = no;
    free(nk); free(src); free(tmpd); free(tmpq); free(tmpk);
    return t;
}

/* Time step of eq. (timestep): min(0.25 h_min/(U + c_s), 0.125 h_min^2/nu). */
double or_timestep(double hmin, double U, double cs, double nu)
{
    double a = 0.25 * (hmin / (U + cs));
    double b = nu > 0.0 ? 0.125 * (hmin * hmin / nu) : a;
    return a < b ? a : b;
}

/* ------------------------------------------------------------------------ */
/* Adaptive refinement (section 3).                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *x, *y, *u, *v, *p, *rho, *h, *mref;
    int64_t* mq;
    int32_t* kind;
    int64_t* origin;
    int32_t* sat;
} or_state;

static void st_copy(or_state* dst, int64_t di, const or_state* src, int64_t si)
{
    dst->x[di] = src->x[si]; dst->y[di] = src->y[si];
    dst->u[di] = src->u[si]; dst->v[di] = src->v[si];
    dst->p[di] = src->p[si]; dst->rho[di] = src->rho[si];
    dst->h[di] = src->h[si]; dst->mref[di] = src->mref[si];
    dst->mq[di] = src->mq[si]; dst->kind[di] = src->kind[si];
    dst->origin[di] = src->origin[si]; dst->sat[di] = src->sat[si];
}

static int alloc_state(or_state* s, int64_t cap)
{
    size_t c = (size_t)(cap > 0 ? cap : 1);
    s->x = malloc(c * 8); s->y = malloc(c * 8); s->u = malloc(c * 8); s->v = malloc(c * 8);
    s->p = malloc(c * 8); s->rho = malloc(c * 8); s->h = malloc(c * 8); s->mref = malloc(c * 8);
    s->mq = malloc(c * 8); s->kind = malloc(c * 4); s->origin = malloc(c * 8); s->sat = malloc(c * 4);
    return s->x && s->y && s->u && s->v && s->p && s->rho && s->h && s->mref && s->mq &&
           s->kind && s->origin && s->sat;
}

static void free_state(or_state* s)
{
    free(s->x); free(s->y); free(s->u); free(s->v); free(s->p); free(s->rho);
    free(s->h); free(s->mref); free(s->mq); free(s->kind); free(s->origin); free(s->sat);
}

/* Split (section 3.1): every fluid particle with m > m_max = mmax_f m_ref is
 * replaced by 7 children: the centre child keeps the parent slot, six are
 * placed at r_p + eps h_p (cos k pi/3, sin k pi/3), k = 0..5, and appended
 * in (parent slot, k) order (READING: canonical slot layout).  Children get
 * h = alpha h_p and copy u, v, p, rho, m_ref.  Mass uses the integer ledger
 * (READING: m = mq q exactly; six children get floor(mq/7), the centre the
 * rest), so total mass is conserved exactly.  Returns the number split. */
static int64_t split_pass(const or_domain* d, const or_params* P, int64_t n,
                          or_state* s, int64_t cap, int64_t* n_out)
{
    static const double ck[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double sk[6] = {0.0, OR_SIN60, OR_SIN60, 0.0, -OR_SIN60, -OR_SIN60};
    int64_t ns = 0;
    for (int64_t i = 0; i < n; ++i) {
        double m = (double)s->mq[i] * P->mass_q;
        if (s->kind[i] == 0 && m > P->mmax_f * s->mref[i]) ++ns;
    }
    if (n + 6 * ns > cap) { *n_out = n + 6 * ns; return -1; }
    int64_t t = n;
    for (int64_t i = 0; i < n; ++i) {
        double m = (double)s->mq[i] * P->mass_q;
        if (!(s->kind[i] == 0 && m > P->mmax_f * s->mref[i])) continue;
        int64_t c = s->mq[i] / 7;
        double r = P->split_eps * s->h[i];
        double hc = P->split_alpha * s->h[i];
        for (int k = 0; k < 6; ++k) {
            st_copy(s, t, s, i);
            s->x[t] = wrap_axis(d, 0, s->x[i] + r * ck[k]);
            s->y[t] = wrap_axis(d, 1, s->y[i] + r * sk[k]);
            s->h[t] = hc;
            s->mq[t] = c;
            s->sat[t] = 1;
            ++t;
        }
        s->mq[i] = s->mq[i] - 6 * c;
        s->h[i] = hc;
    }
    *n_out = t;
    return ns;
}

/* One merge iteration (section 3.2).  closest_i is the allowed j in N(i)
 * with the smallest r_ij^2 (ties to the smaller index).  Allowed: j != i,
 * both fluid, neither has m > m_max (READING: "not identified for
 * splitting", on the current state), r_ij < (h_i + h_j)/2 and
 * m_i + m_j < max(m_max,i, m_max,j).  Mutually closest pairs merge into the
 * smaller index: eq. (merged-pos) and (merged-prop) with mass weights,
 * eq. (merged-h) for h (d = 2); READING: m_ref of the merged particle is the
 * smaller of the two.  Deleted slots are removed by stable compaction. */
static int64_t merge_pass(const or_domain* d, const or_params* P, int64_t n,
                          or_state* s, or_state* tmp, int64_t* n_out)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, s->x, s->y, s->h, &rp, &col);
    if (nnz < 0) return nnz;
    int64_t* closest = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        closest[i] = -1;
        double mi = (double)s->mq[i] * P->mass_q;
        double mmi = P->mmax_f * s->mref[i];
        if (s->kind[i] != 0 || mi > mmi) continue;
        double best = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            if (j == i || s->kind[j] != 0) continue;
            double mj = (double)s->mq[j] * P->mass_q;
            double mmj = P->mmax_f * s->mref[j];
            if (mj > mmj) continue;
            double dx = mi_axis(d, 0, s->x[i] - s->x[j]);
            double dy = mi_axis(d, 1, s->y[i] - s->y[j]);
            double r2 = dx * dx + dy * dy;
            double hh = 0.5 * (s->h[i] + s->h[j]);
            if (!(r2 < hh * hh)) continue;
            double msum = (double)(s->mq[i] + s->mq[j]) * P->mass_q;
            double mm = mmi > mmj ? mmi : mmj;
            if (!(msum < mm)) continue;
            if (closest[i] < 0 || r2 < best) { closest[i] = j; best = r2; }
        }
    }
    free(rp);
    free(col);
    int64_t npairs = 0, t = 0;
    const double w01 = or_w(0.0, 1.0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = closest[i];
        int mutual = (j >= 0 && closest[j] == i);
        if (mutual && j < i) continue; /* deleted: merged into j */
        st_copy(tmp, t, s, i);
        if (mutual) {
            /* a = i (smaller), b = j */
            ++npairs;
            double ma = (double)s->mq[i] * P->mass_q;
            double mb = (double)s->mq[j] * P->mass_q;
            int64_t mqm = s->mq[i] + s->mq[j];
            double mm = (double)mqm * P->mass_q;
            double xb = s->x[i] - mi_axis(d, 0, s->x[i] - s->x[j]);
            double yb = s->y[i] - mi_axis(d, 1, s->y[i] - s->y[j]);
            double xm = (ma * s->x[i] + mb * xb) / mm;
            double ym = (ma * s->y[i] + mb * yb) / mm;
            double dax = xm - s->x[i], day = ym - s->y[i];
            double dbx = xm - xb, dby = ym - yb;
            double ra = sqrt(dax * dax + day * day);
            double rb = sqrt(dbx * dbx + dby * dby);
            double den = ma * or_w(ra, s->h[i]) + mb * or_w(rb, s->h[j]);
            tmp->h[t] = sqrt(mm * w01 / den);
            tmp->x[t] = wrap_axis(d, 0, xm);
            tmp->y[t] = wrap_axis(d, 1, ym);
            tmp->u[t] = (ma * s->u[i] + mb * s->u[j]) / mm;
            tmp->v[t] = (ma * s->v[i] + mb * s->v[j]) / mm;
            tmp->p[t] = (ma * s->p[i] + mb * s->p[j]) / mm;
            tmp->rho[t] = (ma * s->rho[i] + mb * s->rho[j]) / mm;
            tmp->mref[t] = s->mref[i] < s->mref[j] ? s->mref[i] : s->mref[j];
            tmp->mq[t] = mqm;
        }
        ++t;
    }
    free(closest);
    for (int64_t i = 0; i < t; ++i) st_copy(s, i, tmp, i);
    *n_out = t;
    return npairs;
}

/* One shifting iteration after adaptation (section 3.2, last paragraph, and
 * the algorithm of section 3.4): limited Lind shift of every fluid particle
 * (eqs. shift-deltar and shift-limit with rho_0), then the Taylor correction
 * phi' = phi + grad(phi) . dr of eq. (shift-correct).  READING: grad(phi) is
 * the first-order difference form sum_j (m_j/rho_j)(phi_j - phi_i) gradW(h_i)
 * for phi in {u, v, p}, evaluated before moving; density is not corrected. */
static int shift_pass(const or_domain* d, const or_params* P, int64_t n, or_state* s)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, s->x, s->y, s->h, &rp, &col);
    if (nnz < 0) return (int)nnz;
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double* m = malloc(sz);
    for (int64_t i = 0; i < n; ++i) m[i] = (double)s->mq[i] * P->mass_q;
    double *ddx = malloc(sz), *ddy = malloc(sz), *nu = malloc(sz), *nv = malloc(sz), *np = malloc(sz);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (s->kind[i] != 0) { ddx[i] = ddy[i] = 0.0; nu[i] = s->u[i]; nv[i] = s->v[i]; np[i] = s->p[i]; continue; }
        shift_one(d, P->rho0, i, s->x, s->y, s->h, m, rp, col, &ddx[i], &ddy[i]);
        double gux = 0, guy = 0, gvx = 0, gvy = 0, gpx = 0, gpy = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            double dx = mi_axis(d, 0, s->x[i] - s->x[j]);
            double dy = mi_axis(d, 1, s->y[i] - s->y[j]);
            double r = sqrt(dx * dx + dy * dy);
            if (r <= 0.0) continue;
            double f = or_dwdr(r, s->h[i]) / r;
            double wx = f * dx, wy = f * dy;
            double Vj = m[j] / s->rho[j];
            double du = s->u[j] - s->u[i], dv = s->v[j] - s->v[i], dp = s->p[j] - s->p[i];
            gux += Vj * du * wx; guy += Vj * du * wy;
            gvx += Vj * dv * wx; gvy += Vj * dv * wy;
            gpx += Vj * dp * wx; gpy += Vj * dp * wy;
        }
        nu[i] = s->u[i] + (gux * ddx[i] + guy * ddy[i]);
        nv[i] = s->v[i] + (gvx * ddx[i] + gvy * ddy[i]);
        np[i] = s->p[i] + (gpx * ddx[i] + gpy * ddy[i]);
    }
    for (int64_t i = 0; i < n; ++i) {
        s->x[i] = wrap_axis(d, 0, s->x[i] + ddx[i]);
        s->y[i] = wrap_axis(d, 1, s->y[i] + ddy[i]);
        s->u[i] = nu[i]; s->v[i] = nv[i]; s->p[i] = np[i];
    }
    free(m); free(ddx); free(ddy); free(nu); free(nv); free(np);
    free(rp); free(col);
    return OR_OK;
}

/* Smoothing length from the average neighbour mass (section 3.1):
 * h_i = C sqrt(mbar_i / rho_i) with mbar_i the mean mass over N(i), self
 * included, C = h/dx of the run (READING) and rho_i the stored density. */
static int hupdate_pass(const or_domain* d, const or_params* P, int64_t n, or_state* s)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_nbr_cells_alloc(d, n, s->x, s->y, s->h, &rp, &col);
    if (nnz < 0) return (int)nnz;
    double* nh = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (s->kind[i] != 0) { nh[i] = s->h[i]; continue; }
        double sm = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) sm += (double)s->mq[col[k]] * P->mass_q;
        double mbar = sm / (double)(rp[i + 1] - rp[i]);
        nh[i] = P->hdx * sqrt(mbar / s->rho[i]);
    }
    memcpy(s->h, nh, sizeof(double) * (size_t)n);
    free(nh); free(rp); free(col);
    return OR_OK;
}

/* Full adaptation (algorithm of section 3.4, items 5-7): split, merge
 * merge_iters times, shift shift_iters times with the Taylor correction,
 * then set h from the average neighbour mass.  READING: split flags come
 * from the state on entry; children take part in the first merge.
 * Two-phase: if the split would exceed cap, nothing is modified and
 * OR_E_CAPACITY is returned with counts[1] = required size.
 * Outputs: origin[s] = the pre-adaptation slot that slot s descends from;
 * sat[s] = 1 for the six off-centre children; counts = {n_split, n_required,
 * merged pairs per iteration...}.  Returns the new particle count. */
int64_t or_adapt(const or_domain* d, const or_params* P, int64_t n, int64_t cap,
                 double* x, double* y, double* u, double* v, double* p, double* rho,
                 double* h, double* mref, int64_t* mq, int32_t* kind,
                 int64_t* origin, int32_t* sat, int64_t* counts)
{
    or_state s = {x, y, u, v, p, rho, h, mref, mq, kind, origin, sat};
    int32_t* kbuf = NULL;
    if (!kind) {
        kbuf = (int32_t*)calloc((size_t)(cap > 0 ? cap : 1), sizeof(int32_t));
        s.kind = kbuf;
    }
    for (int64_t i = 0; i < n; ++i) { origin[i] = i; sat[i] = 0; }
    int64_t nn = 0;
    /* capacity check before any modification */
    {
        int64_t ns = 0;
        for (int64_t i = 0; i < n; ++i) {
            double m = (double)mq[i] * P->mass_q;
            if (s.kind[i] == 0 && m > P->mmax_f * mref[i]) ++ns;
        }
        counts[0] = ns;
        counts[1] = n + 6 * ns;
        if (n + 6 * ns > cap) { free(kbuf); return OR_E_CAPACITY; }
    }
    split_pass(d, P, n, &s, cap, &nn);
    or_state tmp;
    if (!alloc_state(&tmp, nn)) { free(kbuf); return OR_E_NOMEM; }
    for (int it = 0; it < P->merge_iters; ++it) {
        int64_t n2 = 0;
        int64_t np = merge_pass(d, P, nn, &s, &tmp, &n2);
        if (np < 0) { free_state(&tmp); free(kbuf); return np; }
        counts[2 + it] = np;
        nn = n2;
    }
    free_state(&tmp);
    for (int it = 0; it < P->shift_iters; ++it) {
        int rc = shift_pass(d, P, nn, &s);
        if (rc) { free(kbuf); return rc; }
    }
    int rc = hupdate_pass(d, P, nn, &s);
    free(kbuf);
    if (rc) return rc;
    return nn;
}

/* Stand-alone pieces of the adaptation, for finer-grained pins. */
int64_t or_split_only(const or_domain* d, const or_params* P, int64_t n, int64_t cap,
                      double* x, double* y, double* u, double* v, double* p, double* rho,
                      double* h, double* mref, int64_t* mq, int32_t* kind,
                      int64_t* origin, int32_t* sat)
{
    or_state s = {x, y, u, v, p, rho, h, mref, mq, kind, origin, sat};
    for (int64_t i = 0; i < n; ++i) { origin[i] = i; sat[i] = 0; }
    int64_t nn = 0;
    if (split_pass(d, P, n, &s, cap, &nn) < 0) return OR_E_CAPACITY;
    return nn;
}

int64_t or_merge_only(const or_domain* d, const or_params* P, int64_t n,
                      double* x, double* y, double* u, double* v, double* p, double* rho,
                      double* h, double* mref, int64_t* mq, int32_t* kind,
                      int64_t* origin, int32_t* sat, int64_t* npairs)
{
    or_state s = {x, y, u, v, p, rho, h, mref, mq, kind, origin, sat};
    for (int64_t i = 0; i < n; ++i) { origin[i] = i; sat[i] = 0; }
    or_state tmp;
    if (!alloc_state(&tmp, n)) return OR_E_NOMEM;
    int64_t nn = 0;
    *npairs = merge_pass(d, P, n, &s, &tmp, &nn);
    free_state(&tmp);
    return nn;
}

int or_shift_only(const or_domain* d, const or_params* P, int64_t n,
                  double* x, double* y, double* u, double* v, double* p, double* rho,
                  double* h, double* mref, int64_t* mq, int32_t* kind)
{
    int64_t* o = malloc(8 * (size_t)(n > 0 ? n : 1));
    int32_t* st = malloc(4 * (size_t)(n > 0 ? n : 1));
    or_state s = {x, y, u, v, p, rho, h, mref, mq, kind, o, st};
    int rc = shift_pass(d, P, n, &s);
    free(o); free(st);
    return rc;
}

int or_hupdate_only(const or_domain* d, const or_params* P, int64_t n,
                    double* x, double* y, double* rho, double* h, int64_t* mq, int32_t* kind)
{
    or_state s;
    memset(&s, 0, sizeof(s));
    s.x = x; s.y = y; s.rho = rho; s.h = h; s.mq = mq; s.kind = kind;
    return hupdate_pass(d, P, n, &s);
}

/* ------------------------------------------------------------------------ */
/* Background particles (section 3.3).                                       */
/* ------------------------------------------------------------------------ */

/* Fluid reference mass from the background (algorithm of section 3.4,
 * item 4, and section 3.3): the minimum m_ref over background particles
 * within the symmetric support 3 max(h_i, h_b).  READING: if none is in
 * range, the nearest background particle (ties to the smaller index). */
int or_mref_lookup(const or_domain* d, int64_t n, const double* x, const double* y,
                   const double* h, int64_t nb, const double* bx, const double* by,
                   const double* bh, const double* bmref, double* mref)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_xnbr_cells_alloc(d, n, x, y, h, nb, bx, by, bh, &rp, &col);
    if (nnz < 0) return (int)nnz;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] > rp[i]) {
            double mn = bmref[col[rp[i]]];
            for (int64_t k = rp[i] + 1; k < rp[i + 1]; ++k)
                if (bmref[col[k]] < mn) mn = bmref[col[k]];
            mref[i] = mn;
        } else {
            int64_t best = -1;
            double br = 0.0;
            for (int64_t b = 0; b < nb; ++b) {
                double dx = mi_axis(d, 0, x[i] - bx[b]);
                double dy = mi_axis(d, 1, y[i] - by[b]);
                double r2 = dx * dx + dy * dy;
                if (best < 0 || r2 < br) { best = b; br = r2; }
            }
            if (best >= 0) mref[i] = bmref[best];
        }
    }
    free(rp);
    free(col);
    return OR_OK;
}

/* One background pass, steps 1-4 of section 3.3.
 * Step 1: mask_b = 1 and ds_b = ds_min where a solid particle is within
 *   3 max(h_b, h_s); also where the background particle carries the
 *   solution mark (the solution-adaptivity rule of section 3.3): in the
 *   first pass of an update the mark (mask bit 2) is set where phi_b >
 *   phi_thresh (cleared everywhere when phi is not given); later passes and
 *   split children keep it.  READING: the paper marks these particles once
 *   per update and lets the rest of the algorithm proceed, so the mark
 *   lasts the whole update.  mask is 0, 1 (near a body) or 3 (marked).
 * Step 2 (Jacobi, self included): for unmasked b, with min, max and
 *   geometric mean of ds over N(b): ds' = C_r min if max/min < C_r^3, else
 *   the geometric mean; READING: clamped to [ds_min, ds_max].
 *   m_ref = rho_0 ds^2.
 * Step 3: split background particles with mass > mmax_f m_ref (same split).
 * Step 4, smooth_iters times on a fresh N(b): h from eq. (h-smoothing) and
 *   the Lind shift (eq. shift-deltar, volume m_b / rho_0), both from the
 *   same neighbour set, applied together.
 * Returns the new background count or a negative error. */
/* Exact sum of doubles, rounded once (a long accumulator).  Every finite
 * double is an integer multiple of 2^-1074, so a sum of them is V 2^-1074
 * with V an integer; V is held in base-2^32 digits (int64 cells with room
 * for the carries of 2^30 additions), and the result is V rounded to 53
 * significant bits, ties to even, times 2^-1074: the correctly rounded sum,
 * the same whatever the order of the terms.
 * READING: the background update's sums over neighbours (the logarithms of
 * the sizes in the grading, h_j and the shift terms in the smoothing) are set
 * sums.  They are taken correctly rounded, so that the update is a function
 * of the particle set alone, whatever the slot order: near-cancelling shift
 * terms (a particle on a symmetry line) round differently in different
 * orders even when compensated, and the repeated update can amplify that. */
#define OR_XS_N 70
typedef struct { int64_t d[OR_XS_N]; } or_xsum;

static void xsum_init(or_xsum* a) { memset(a->d, 0, sizeof(a->d)); }

static void xsum_add(or_xsum* a, double x)
{
    if (x == 0.0) return;
    uint64_t bits;
    memcpy(&bits, &x, sizeof(bits));
    int neg = (int)(bits >> 63);
    int E = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & ((1ull << 52) - 1);
    int p = 0;                   /* x = m 2^(p - 1074) */
    if (E > 0) { m |= 1ull << 52; p = E - 1; }
    int k = p / 32, sft = p % 32;
    uint64_t lo = (m & 0xffffffffull) << sft;  /* < 2^63 */
    uint64_t hi = (m >> 32) << sft;            /* < 2^52 */
    int64_t c0 = (int64_t)(lo & 0xffffffffull);
    int64_t c1 = (int64_t)(lo >> 32) + (int64_t)(hi & 0xffffffffull);
    int64_t c2 = (int64_t)(hi >> 32);
    if (neg) { c0 = -c0; c1 = -c1; c2 = -c2; }
    a->d[k] += c0;
    a->d[k + 1] += c1;
    a->d[k + 2] += c2;
}

/* digits to [0, 2^32) from the bottom up, the top cell keeping the sign */
static void xsum_carry(int64_t* d)
{
    for (int k = 0; k < OR_XS_N - 1; ++k) {
        int64_t c = d[k] >> 32;  /* floor(d / 2^32) */
        d[k] -= c * 4294967296LL;
        d[k + 1] += c;
    }
}

static int xsum_bit(const int64_t* d, int i) { return (int)((d[i / 32] >> (i % 32)) & 1); }

static double xsum_get(const or_xsum* a)
{
    int64_t d[OR_XS_N];
    memcpy(d, a->d, sizeof(d));
    xsum_carry(d);
    int neg = d[OR_XS_N - 1] < 0;
    if (neg) {  /* |V| */
        for (int k = 0; k < OR_XS_N; ++k) d[k] = -d[k];
        xsum_carry(d);
    }
    int nb = 0;  /* bit length of |V| */
    for (int i = 32 * OR_XS_N - 1; i >= 0; --i)
        if (xsum_bit(d, i)) { nb = i + 1; break; }
    if (nb == 0) return 0.0;
    int drop = nb > 53 ? nb - 53 : 0;
    double t = 0.0;  /* the kept 53 (or fewer) bits, exact */
    for (int i = nb - 1; i >= drop; --i) t = 2.0 * t + (double)xsum_bit(d, i);
    if (drop > 0 && xsum_bit(d, drop - 1)) {
        int sticky = 0;
        for (int i = 0; i < drop - 1 && !sticky; ++i) sticky = xsum_bit(d, i);
        if (sticky || fmod(t, 2.0) == 1.0) t += 1.0;  /* above half, or a tie to even */
    }
    double r = ldexp(t, drop - 1074);
    return neg ? -r : r;
}

/* The exact sum of n doubles, rounded once (pinned against Python's
 * correctly rounded math.fsum). */
double or_exact_sum(int64_t n, const double* x)
{
    or_xsum a;
    xsum_init(&a);
    for (int64_t i = 0; i < n; ++i) xsum_add(&a, x[i]);
    return xsum_get(&a);
}

/* The limited shift of background particle b (eqs. shift-deltar and
 * shift-limit, the same terms as shift_one) with the sums correctly
 * rounded. */
static void bg_shift_one(const or_domain* d, double rho0, int64_t b, const double* x,
                         const double* y, const double* h, const double* m,
                         const int64_t* rp, const int32_t* col, double* dxs, double* dys)
{
    double fxi = or_kf(OR_XI);
    or_xsum sx, sy;
    xsum_init(&sx);
    xsum_init(&sy);
    for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
        int64_t j = col[k];
        double dx = mi_axis(d, 0, x[b] - x[j]);
        double dy = mi_axis(d, 1, y[b] - y[j]);
        double r = sqrt(dx * dx + dy * dy);
        if (r <= 0.0) continue;
        double hij = 0.5 * (h[b] + h[j]);
        double wr = or_kf(r / hij) / fxi;
        double coef = (m[j] / rho0) * (1.0 + 0.24 * ((wr * wr) * (wr * wr)));
        double t = coef * (or_dwdr(r, hij) / r);
        xsum_add(&sx, t * dx);
        xsum_add(&sy, t * dy);
    }
    double pref = -0.5 * (h[b] * h[b]);
    double ddx = pref * xsum_get(&sx), ddy = pref * xsum_get(&sy);
    double mag = sqrt(ddx * ddx + ddy * ddy);
    double lim = 0.25 * h[b];
    if (mag > lim) {
        double th = lim / mag;
        ddx = ddx * th;
        ddy = ddy * th;
    }
    *dxs = ddx;
    *dys = ddy;
}

static int64_t bg_one_pass(const or_domain* d, const or_bgparams* B, int64_t nb, int64_t cap,
                           double* bx, double* by, double* bh, double* bds, int32_t* bmask,
                           int64_t* bmq, double* bmref, int64_t ns, const double* sx,
                           const double* sy, const double* sh, const double* phi,
                           double phi_thresh, int first, int64_t* nsplit)
{
    int64_t *rp = NULL;
    int32_t *col = NULL;
    size_t sz8 = sizeof(double) * (size_t)(nb > 0 ? nb : 1);
    /* step 1 */
    int64_t nnz = or_xnbr_cells_alloc(d, nb, bx, by, bh, ns, sx, sy, sh, &rp, &col);
    if (nnz < 0) return nnz;
    for (int64_t b = 0; b < nb; ++b) {
        int sol = first ? ((phi && phi[b] > phi_thresh) ? 2 : 0) : (bmask[b] & 2);
        int m = rp[b + 1] > rp[b] ? 1 : 0;
        if (sol) m |= 3;
        bmask[b] = m;
        if (m) bds[b] = B->ds_min;
    }
    free(rp); free(col);
    /* step 2 */
    nnz = or_nbr_cells_alloc(d, nb, bx, by, bh, &rp, &col);
    if (nnz < 0) return nnz;
    double* nds = malloc(sz8);
    double cr3 = B->cr * B->cr * B->cr;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t b = 0; b < nb; ++b) {
        if (bmask[b]) { nds[b] = bds[b]; continue; }
        double mn = bds[col[rp[b]]], mx = mn;
        or_xsum sl;
        xsum_init(&sl);
        for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
            double s = bds[col[k]];
            if (s < mn) mn = s;
            if (s > mx) mx = s;
            xsum_add(&sl, log(s));
        }
        double geo = exp(xsum_get(&sl) / (double)(rp[b + 1] - rp[b]));
        double nv = (mx / mn < cr3) ? B->cr * mn : geo;
        if (nv < B->ds_min) nv = B->ds_min;
        if (nv > B->ds_max) nv = B->ds_max;
        nds[b] = nv;
    }
    for (int64_t b = 0; b < nb; ++b) {
        bds[b] = nds[b];
        bmref[b] = B->rho0 * (bds[b] * bds[b]);
    }
    free(nds); free(rp); free(col);
    /* step 3: split */
    int64_t cnt = 0;
    for (int64_t b = 0; b < nb; ++b)
        if ((double)bmq[b] * B->mass_q > B->mmax_f * bmref[b]) ++cnt;
    if (nb + 6 * cnt > cap) return OR_E_CAPACITY;
    {
        static const double ck[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
        const double sk[6] = {0.0, OR_SIN60, OR_SIN60, 0.0, -OR_SIN60, -OR_SIN60};
        int64_t t = nb;
        for (int64_t b = 0; b < nb; ++b) {
            if (!((double)bmq[b] * B->mass_q > B->mmax_f * bmref[b])) continue;
            int64_t c = bmq[b] / 7;
            double r = B->split_eps * bh[b];
            double hc = B->split_alpha * bh[b];
            for (int k = 0; k < 6; ++k) {
                bx[t] = wrap_axis(d, 0, bx[b] + r * ck[k]);
                by[t] = wrap_axis(d, 1, by[b] + r * sk[k]);
                bh[t] = hc;
                bds[t] = bds[b];
                bmask[t] = bmask[b];
                bmref[t] = bmref[b];
                bmq[t] = c;
                ++t;
            }
            bmq[b] = bmq[b] - 6 * c;
            bh[b] = hc;
        }
        *nsplit += cnt;
        nb = t;
    }
    /* step 4 */
    sz8 = sizeof(double) * (size_t)(nb > 0 ? nb : 1);
    double* m = malloc(sz8);
    double *nh = malloc(sz8), *ddx = malloc(sz8), *ddy = malloc(sz8);
    for (int it = 0; it < B->smooth_iters; ++it) {
        for (int64_t b = 0; b < nb; ++b) m[b] = (double)bmq[b] * B->mass_q;
        nnz = or_nbr_cells_alloc(d, nb, bx, by, bh, &rp, &col);
        if (nnz < 0) { free(m); free(nh); free(ddx); free(ddy); return nnz; }
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t b = 0; b < nb; ++b) {
            double N = (double)(rp[b + 1] - rp[b]);
            or_xsum sh_;
            xsum_init(&sh_);
            for (int64_t k = rp[b]; k < rp[b + 1]; ++k) xsum_add(&sh_, bh[col[k]]);
            nh[b] = 0.5 * ((bh[b] / 2.0) * (1.0 + sqrt(B->n_r / N)) + xsum_get(&sh_) / N);
            bg_shift_one(d, B->rho0, b, bx, by, bh, m, rp, col, &ddx[b], &ddy[b]);
        }
        for (int64_t b = 0; b < nb; ++b) {
            bh[b] = nh[b];
            bx[b] = wrap_axis(d, 0, bx[b] + ddx[b]);
            by[b] = wrap_axis(d, 1, by[b] + ddy[b]);
        }
        free(rp); free(col);
    }
    free(m); free(nh); free(ddx); free(ddy);
    return nb;
}

int64_t or_bg_update(const or_domain* d, const or_bgparams* B, int64_t nb, int64_t cap,
                     double* bx, double* by, double* bh, double* bds, int32_t* bmask,
                     int64_t* bmq, double* bmref, int64_t ns, const double* sx,
                     const double* sy, const double* sh, const double* phi,
                     double phi_thresh, int32_t passes, int64_t* nsplit)
{
    *nsplit = 0;
    for (int it = 0; it < passes; ++it) {
        int64_t r = bg_one_pass(d, B, nb, cap, bx, by, bh, bds, bmask, bmq, bmref, ns, sx,
                                sy, sh, it == 0 ? phi : NULL, phi_thresh, it == 0, nsplit);
        if (r < 0) return r;
        nb = r;
    }
    return nb;
}

/* Vorticity magnitude used by solution adaptivity (section 3.3):
 * omega_i = sum_j (m_j/rho_j) [(v_j - v_i) dW/dx - (u_j - u_i) dW/dy] at h_i.
 * Pinned by closed forms: 2 Omega for a rigid rotation, the Taylor-Green
 * vorticity 4 pi cos(2 pi x) cos(2 pi y), and 0 for a uniform translation. */
void or_vorticity(const or_domain* d, int64_t n, const double* x, const double* y,
                  const double* u, const double* v, const double* h, const double* m,
                  const double* rho, const int64_t* rp, const int32_t* col, double* omega)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            double dx = mi_axis(d, 0, x[i] - x[j]);
            double dy = mi_axis(d, 1, y[i] - y[j]);
            double r = sqrt(dx * dx + dy * dy);
            if (r <= 0.0) continue;
            double f = or_dwdr(r, h[i]) / r;
            double Vj = m[j] / rho[j];
            s += Vj * ((v[j] - v[i]) * (f * dx) - (u[j] - u[i]) * (f * dy));
        }
        omega[i] = s;
    }
}

/* Solution adaptivity (section 3.3): a fluid field f (|vorticity|) carried
 * to the background particles by the Shepard average of eq. (shepard),
 * phi_b = sum_i f_i W(r_bi, h_bi) / sum_i W(r_bi, h_bi) with
 * h_bi = (h_b + h_i)/2 over the fluid particles i with
 * r_bi < 3 max(h_b, h_i) (kind 0 only when kind is given); 0 when none.
 * READING: the paper says the field is interpolated onto the background
 * without naming the operator; the Shepard form is the one section 2.2
 * uses for the same purpose. */
int or_shepard_to_bg(const or_domain* d, int64_t nb, const double* bx, const double* by,
                     const double* bh, int64_t n, const double* x, const double* y,
                     const double* h, const int32_t* kind, const double* f, double* phi)
{
    int64_t* rp = NULL;
    int32_t* col = NULL;
    int64_t nnz = or_xnbr_cells_alloc(d, nb, bx, by, bh, n, x, y, h, &rp, &col);
    if (nnz < 0) return (int)nnz;
    for (int64_t b = 0; b < nb; ++b) {
        double S = 0.0, sf = 0.0;
        for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
            int64_t i = col[k];
            if (kind && kind[i] != 0) continue;
            double dx = mi_axis(d, 0, bx[b] - x[i]);
            double dy = mi_axis(d, 1, by[b] - y[i]);
            double r = sqrt(dx * dx + dy * dy);
            double w = or_w(r, 0.5 * (bh[b] + h[i]));
            S += w;
            sf += f[i] * w;
        }
        phi[b] = S > 0.0 ? sf / S : 0.0;
    }
    free(rp);
    free(col);
    return OR_OK;
}
