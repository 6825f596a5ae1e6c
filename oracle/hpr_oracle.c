/*
 * CPU FP64 oracle of the restarted Halpern-Peaceman-Rachford LP iteration.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library; the GPU solver never
 * does, and the two share no source.
 *
 * Problem (the paper's eq.(lp) with two-sided rows):
 *     min c^T x + off  s.t.  lo <= A x <= hi,  l <= x <= u.
 * With hi = +inf a row is the paper's  a_i^T x >= theta_i.
 *
 * Steps, in the paper's order (Section III):
 *   1. scaling: optional Ruiz equilibration, Pock-Chambolle diagonal scaling with
 *      alpha = 1, then normalisation of the bound and cost vectors (Section III-A);
 *   2. lambda = lambda_max(A A^T) of the scaled matrix by the power method;
 *   3. the iteration eq.(hpr): primal projection step with sigma, dual projection
 *      step with 1/(lambda sigma) on A(2 xbar - x), Peaceman-Rachford reflection
 *      and Halpern averaging towards the anchor (x0, y0);
 *   4. every check_every iterations: KKT residuals of (xbar, ybar, zbar) on the
 *      original problem (the residual map R of Theorem 1, normalised), the M-norm
 *      fixed-point residual, restart of the anchor and adaptation of sigma
 *      (the paper names both without giving the rules; the rules here are the
 *      ones written out in the function comments and taken identically by the GPU).
 *
 * The dual projection for a two-sided row: with v = y - s (A xhat),
 *   ybar = v + s lo   if that is > 0,
 *          v + s hi   if that is < 0,
 *          0          otherwise,
 * which for hi = +inf is exactly Pi_{R+}(y + s(theta - A xhat)) of eq.(hpr).
 *
 * Plain loops, FP64 throughout. Row loops of matrix-vector products may run on
 * several OpenMP threads (each row is summed by one thread in index order, so the
 * result does not depend on the thread count); every reduction is serial.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const double *row_lo, *row_hi, *col_lo, *col_hi, *c;
    double obj_offset;
} orc_lp;

typedef struct {
    double tol;              /* stop when rel_kkt <= tol (0: never) */
    int64_t max_iter;        /* >= 1 */
    int32_t check_every;     /* >= 1 */
    int32_t ruiz_iters;      /* 0: off */
    int32_t use_pc;          /* Pock-Chambolle, alpha = 1 */
    int32_t use_bc;          /* bound/cost normalisation */
    int32_t restart;         /* restart rule on/off */
    int32_t sigma_update;    /* sigma adaptation on/off */
    double sigma0;
    double lambda_in;        /* > 0: use this lambda, skip the power method */
    uint64_t seed;           /* power-method start vector */
    int32_t power_max_iter;
    double power_tol;
    double time_limit;       /* seconds, <= 0: none */
    double sigma_smoothing;  /* weight w of sigma* in log sigma <- (1 - w) log sigma + w log sigma* */
    double sigma_smoothing_warm;  /* the same weight when a start point (x0 or y0) is given */
    const double *x0;        /* warm start (original space) or NULL */
    const double *y0;
} orc_opts;

typedef struct {
    int32_t term;            /* 1 solved, 2 iteration limit, 3 time limit, 4 numeric failure,
                                5 primal infeasible, 6 dual infeasible (no finite optimum) */
    int64_t iters, restarts;
    double pobj, dobj, rel_p, rel_d, rel_gap, rel_kkt, lambda, sigma, setup_s, solve_s;
} orc_info;

enum { ORC_SOLVED = 1, ORC_ITER_LIMIT = 2, ORC_TIME_LIMIT = 3, ORC_NUMERIC_FAIL = 4, ORC_PRIMAL_INFEASIBLE = 5,
       ORC_DUAL_INFEASIBLE = 6 };

/* relative margin of the primal infeasibility certificate */
#define ORC_INFEAS_TOL 1e-6

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* ---------------------------------------------------------------- basic algebra */

/* y = A x (rows split over threads only for large matrices; a row is always summed by one
   thread in index order, so the result does not depend on the split) */
static void spmv(int32_t m, const int64_t *rp, const int32_t *ci, const double *v,
                 const double *x, double *y) {
    #pragma omp parallel for schedule(static) if (m > 20000)
    for (int32_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

/* explicit transpose (CSR of A^T); within a column, entries keep increasing row order */
static void transpose(int32_t m, int32_t n, const int64_t *rp, const int32_t *ci, const double *v,
                      int64_t *trp, int32_t *tci, double *tv) {
    int64_t nnz = rp[m];
    memset(trp, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, trp, sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t d = fill[ci[k]]++;
            tci[d] = i;
            tv[d] = v[k];
        }
    free(fill);
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* the finite side of a row's bounds (larger magnitude if both are finite, 0 if none) */
static double finite_side(double lo, double hi) {
    int fl = isfinite(lo), fh = isfinite(hi);
    if (fl && fh) return fabs(lo) > fabs(hi) ? lo : hi;
    if (fl) return lo;
    if (fh) return hi;
    return 0.0;
}

/* ---------------------------------------------------------------- validation */

int orc_validate(const orc_lp *lp) {
    if (!lp || lp->m < 0 || lp->n < 1 || lp->nnz < 0) return -1;
    if (lp->m > 0 && (!lp->row_ptr || !lp->row_lo || !lp->row_hi)) return -1;
    if (!lp->col_lo || !lp->col_hi || !lp->c) return -1;
    if (lp->nnz > 0 && (!lp->col_idx || !lp->val)) return -1;
    if (lp->m > 0) {
        if (lp->row_ptr[0] != 0 || lp->row_ptr[lp->m] != lp->nnz) return -1;
        for (int32_t i = 0; i < lp->m; ++i)
            if (lp->row_ptr[i + 1] < lp->row_ptr[i]) return -1;
    } else if (lp->nnz != 0) {
        return -1;
    }
    if (!isfinite(lp->obj_offset)) return -1;
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)lp->n);
    for (int32_t j = 0; j < lp->n; ++j) mark[j] = -1;
    int bad = 0;
    for (int32_t i = 0; i < lp->m && !bad; ++i)
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
            int32_t j = lp->col_idx[k];
            if (j < 0 || j >= lp->n || !isfinite(lp->val[k]) || mark[j] == i) { bad = 1; break; }
            mark[j] = i;
        }
    free(mark);
    if (bad) return -1;
    for (int32_t i = 0; i < lp->m; ++i) {
        double lo = lp->row_lo[i], hi = lp->row_hi[i];
        if (isnan(lo) || isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY) return -1;
    }
    for (int32_t j = 0; j < lp->n; ++j) {
        double lo = lp->col_lo[j], hi = lp->col_hi[j];
        if (isnan(lo) || isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY) return -1;
        if (!isfinite(lp->c[j])) return -1;
    }
    return 0;
}

/* ---------------------------------------------------------------- KKT of the original problem */

/*
 * Relative KKT residuals of (x, y, z) for min c^T x, lo <= Ax <= hi, l <= x <= u:
 *   rel_p = ||max(lo - Ax, 0, Ax - hi)|| / (1 + ||b||), b = finite sides of the rows;
 *   rel_d = ||c - A^T y - z|| / (1 + ||c||);
 *   pobj = c^T x + off,
 *   dobj = sum_i (lo_i y_i+ - hi_i y_i-) + sum_j (l_j z_j+ - u_j z_j-) + off  (0 * inf = 0);
 *   rel_gap = |pobj - dobj| / (1 + |pobj| + |dobj|)  (1 if dobj is infinite);
 *   rel_kkt = max(rel_p, rel_d, rel_gap).
 * out[0..7] = rel_p, rel_d, rel_gap, rel_kkt, pobj, dobj, ||R|| (Theorem 1 map), unused.
 * The residual map R: (Ax - Pi_[lo,hi](Ax - y); x - Pi_K(x - z); c - A^T y - z); for
 * hi = +inf its first block equals the paper's y - Pi_+(y - Ax + theta).
 */
int orc_kkt(const orc_lp *lp, const double *x, const double *y, const double *z, double *out) {
    int32_t m = lp->m, n = lp->n;
    double *ax = (double *)calloc((size_t)m + 1, sizeof(double));
    double *aty = (double *)calloc((size_t)n, sizeof(double));
    spmv(m, lp->row_ptr, lp->col_idx, lp->val, x, ax);
    for (int32_t i = 0; i < m; ++i)
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k)
            aty[lp->col_idx[k]] += lp->val[k] * y[i];
    double rp2 = 0.0, b2 = 0.0, R2 = 0.0, dobj = lp->obj_offset;
    int dinf = 0;
    for (int32_t i = 0; i < m; ++i) {
        double lo = lp->row_lo[i], hi = lp->row_hi[i], a = ax[i];
        double r = 0.0;
        if (lo - a > r) r = lo - a;
        if (a - hi > r) r = a - hi;
        rp2 += r * r;
        double b = finite_side(lo, hi);
        b2 += b * b;
        double yp = y[i] > 0 ? y[i] : 0.0, ym = y[i] < 0 ? -y[i] : 0.0;
        if (yp > 0) { if (isfinite(lo)) dobj += lo * yp; else dinf = 1; }
        if (ym > 0) { if (isfinite(hi)) dobj -= hi * ym; else dinf = 1; }
        double r1 = a - clampd(a - y[i], lo, hi);
        R2 += r1 * r1;
    }
    double rd2 = 0.0, c2 = 0.0, pobj = lp->obj_offset;
    for (int32_t j = 0; j < n; ++j) {
        double r = lp->c[j] - aty[j] - z[j];
        rd2 += r * r;
        c2 += lp->c[j] * lp->c[j];
        pobj += lp->c[j] * x[j];
        double l = lp->col_lo[j], u = lp->col_hi[j];
        double zp = z[j] > 0 ? z[j] : 0.0, zm = z[j] < 0 ? -z[j] : 0.0;
        if (zp > 0) { if (isfinite(l)) dobj += l * zp; else dinf = 1; }
        if (zm > 0) { if (isfinite(u)) dobj -= u * zm; else dinf = 1; }
        double r2 = x[j] - clampd(x[j] - z[j], l, u);
        R2 += r2 * r2 + r * r;
    }
    double rel_p = sqrt(rp2) / (1.0 + sqrt(b2));
    double rel_d = sqrt(rd2) / (1.0 + sqrt(c2));
    double rel_gap = dinf ? 1.0 : fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
    double rel_kkt = rel_p;
    if (rel_d > rel_kkt) rel_kkt = rel_d;
    if (rel_gap > rel_kkt) rel_kkt = rel_gap;
    if (isnan(rel_p) || isnan(rel_d) || isnan(rel_gap)) rel_kkt = NAN;
    out[0] = rel_p; out[1] = rel_d; out[2] = rel_gap; out[3] = rel_kkt;
    out[4] = pobj; out[5] = dinf ? -INFINITY : dobj; out[6] = sqrt(R2); out[7] = 0.0;
    free(ax);
    free(aty);
    return 0;
}

/* ---------------------------------------------------------------- scaling */

typedef struct {
    int32_t m, n;
    int64_t *rp, *trp;
    int32_t *ci, *tci;
    double *v, *tv;           /* scaled A and its transpose */
    double *lo, *hi, *l, *u, *c;
    double *dr, *dc;          /* x = beta_b dc xs, y = beta_c dr ys, z = beta_c zs / dc */
    double beta_b, beta_c;
} scaled_lp;

static void free_scaled(scaled_lp *s) {
    free(s->rp); free(s->trp); free(s->ci); free(s->tci); free(s->v); free(s->tv);
    free(s->lo); free(s->hi); free(s->l); free(s->u); free(s->c); free(s->dr); free(s->dc);
}

static void apply_diag(scaled_lp *s, const double *er, const double *ec) {
    for (int32_t i = 0; i < s->m; ++i)
        for (int64_t k = s->rp[i]; k < s->rp[i + 1]; ++k) s->v[k] *= er[i] * ec[s->ci[k]];
    for (int32_t i = 0; i < s->m; ++i) s->dr[i] *= er[i];
    for (int32_t j = 0; j < s->n; ++j) s->dc[j] *= ec[j];
}

/*
 * Ruiz passes (optional): divide each row and column by the square root of its
 * largest magnitude. Pock-Chambolle, alpha = 1: divide each row by the square root
 * of its absolute row sum and each column by the square root of its absolute
 * column sum (empty rows/columns keep factor 1). Then the scaled problem is
 *   A~ = Dr A Dc,  Dr lo <= A~ xs <= Dr hi,  l / Dc <= xs <= u / Dc,  cost Dc c,
 * and the normalisation divides bounds by beta_b = 1 + ||b~|| (b~ the finite sides
 * of the scaled rows) and the cost by beta_c = 1 + ||c~||.
 */
static void build_scaled(const orc_lp *lp, const orc_opts *o, scaled_lp *s) {
    int32_t m = lp->m, n = lp->n;
    int64_t nnz = lp->nnz;
    s->m = m; s->n = n;
    s->rp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
    s->ci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    s->v = (double *)malloc(sizeof(double) * ((size_t)nnz + 1));
    if (m > 0) memcpy(s->rp, lp->row_ptr, sizeof(int64_t) * ((size_t)m + 1)); else s->rp[0] = 0;
    if (nnz) {
        memcpy(s->ci, lp->col_idx, sizeof(int32_t) * (size_t)nnz);
        memcpy(s->v, lp->val, sizeof(double) * (size_t)nnz);
    }
    s->dr = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    s->dc = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < m; ++i) s->dr[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) s->dc[j] = 1.0;
    double *er = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    double *ec = (double *)malloc(sizeof(double) * (size_t)n);

    for (int32_t it = 0; it < o->ruiz_iters; ++it) {
        for (int32_t j = 0; j < n; ++j) ec[j] = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            double r = 0.0;
            for (int64_t k = s->rp[i]; k < s->rp[i + 1]; ++k) {
                double a = fabs(s->v[k]);
                if (a > r) r = a;
                if (a > ec[s->ci[k]]) ec[s->ci[k]] = a;
            }
            er[i] = r > 0 ? 1.0 / sqrt(r) : 1.0;
        }
        for (int32_t j = 0; j < n; ++j) ec[j] = ec[j] > 0 ? 1.0 / sqrt(ec[j]) : 1.0;
        apply_diag(s, er, ec);
    }
    if (o->use_pc) {
        for (int32_t j = 0; j < n; ++j) ec[j] = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            double r = 0.0;
            for (int64_t k = s->rp[i]; k < s->rp[i + 1]; ++k) {
                r += fabs(s->v[k]);
                ec[s->ci[k]] += fabs(s->v[k]);
            }
            er[i] = r > 0 ? 1.0 / sqrt(r) : 1.0;
        }
        for (int32_t j = 0; j < n; ++j) ec[j] = ec[j] > 0 ? 1.0 / sqrt(ec[j]) : 1.0;
        apply_diag(s, er, ec);
    }
    free(er);
    free(ec);

    s->lo = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    s->hi = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    s->l = (double *)malloc(sizeof(double) * (size_t)n);
    s->u = (double *)malloc(sizeof(double) * (size_t)n);
    s->c = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < m; ++i) { s->lo[i] = lp->row_lo[i] * s->dr[i]; s->hi[i] = lp->row_hi[i] * s->dr[i]; }
    for (int32_t j = 0; j < n; ++j) {
        s->l[j] = lp->col_lo[j] / s->dc[j];
        s->u[j] = lp->col_hi[j] / s->dc[j];
        s->c[j] = lp->c[j] * s->dc[j];
    }
    s->beta_b = 1.0;
    s->beta_c = 1.0;
    if (o->use_bc) {
        double b2 = 0.0;
        for (int32_t i = 0; i < m; ++i) { double b = finite_side(s->lo[i], s->hi[i]); b2 += b * b; }
        s->beta_b = 1.0 + sqrt(b2);
        s->beta_c = 1.0 + nrm2(n, s->c);
        for (int32_t i = 0; i < m; ++i) { s->lo[i] /= s->beta_b; s->hi[i] /= s->beta_b; }
        for (int32_t j = 0; j < n; ++j) { s->l[j] /= s->beta_b; s->u[j] /= s->beta_b; s->c[j] /= s->beta_c; }
    }
    s->trp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    s->tci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    s->tv = (double *)malloc(sizeof(double) * ((size_t)nnz + 1));
    transpose(m, n, s->rp, s->ci, s->v, s->trp, s->tci, s->tv);
}

/* ---------------------------------------------------------------- power method */

/* SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014), used as a counter-based generator:
   draw i is mix(seed + (i + 1) * golden gamma). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [-1, 1): 53 high bits */
double orc_start_value(uint64_t seed, uint64_t i) {
    return 2.0 * ((double)(splitmix64_at(seed, i) >> 11) * 0x1.0p-53) - 1.0;
}

/*
 * lambda_max(A~ A~^T) by the power method: v <- A~(A~^T v) / ||.||, estimate ||A~ A~^T v||
 * for unit v; stop when the estimate changes by at most tol (relative) or after
 * max_iter products. Returned lambda = 1.01 * estimate, capped at 1 when the
 * Pock-Chambolle scaling is on (it bounds ||A~|| by 1), and 1 when the estimate is 0.
 */
static double power_lambda(const scaled_lp *s, const orc_opts *o, int32_t *iters_out) {
    int32_t m = s->m, n = s->n;
    if (m == 0 || s->rp[m] == 0) { if (iters_out) *iters_out = 0; return 1.0; }
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
    double *w = (double *)malloc(sizeof(double) * (size_t)m);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < m; ++i) v[i] = orc_start_value(o->seed, (uint64_t)i);
    double nv = nrm2(m, v);
    for (int32_t i = 0; i < m; ++i) v[i] /= nv;
    double est = 0.0, prev = 0.0;
    int32_t it = 0;
    for (it = 1; it <= o->power_max_iter; ++it) {
        spmv(n, s->trp, s->tci, s->tv, v, t);
        spmv(m, s->rp, s->ci, s->v, t, w);
        est = nrm2(m, w);
        if (est == 0.0) break;
        for (int32_t i = 0; i < m; ++i) v[i] = w[i] / est;
        if (it > 1 && fabs(est - prev) <= o->power_tol * est) break;
        prev = est;
    }
    if (it > o->power_max_iter) it = o->power_max_iter;
    free(v); free(w); free(t);
    if (iters_out) *iters_out = it;
    if (est == 0.0) return 1.0;
    double lam = 1.01 * est;
    if (o->use_pc && lam > 1.0) lam = 1.0;
    return lam;
}

/* Scaled data for tests: dr[m], dc[n], out[0..3] = beta_b, beta_c, lambda, power iterations. */
int orc_scaling(const orc_lp *lp, const orc_opts *o, double *dr, double *dc, double *out) {
    if (orc_validate(lp)) return -1;
    scaled_lp s;
    build_scaled(lp, o, &s);
    memcpy(dr, s.dr, sizeof(double) * (size_t)lp->m);
    memcpy(dc, s.dc, sizeof(double) * (size_t)lp->n);
    int32_t pit = 0;
    out[0] = s.beta_b;
    out[1] = s.beta_c;
    out[2] = o->lambda_in > 0 ? o->lambda_in : power_lambda(&s, o, &pit);
    out[3] = pit;
    free_scaled(&s);
    return 0;
}

/* ---------------------------------------------------------------- one iteration of eq.(hpr) */

/*
 * One step of eq.(hpr) on the problem as given (no scaling), from (x, y) with anchor
 * (x0, y0) and inner counter k. Outputs the bar point (xb, yb, zb) and overwrites
 * x, y with the averaged iterate. lambda and sigma as given.
 */
static void hpr_step(int32_t m, int32_t n,
                     const int64_t *rp, const int32_t *ci, const double *v,
                     const int64_t *trp, const int32_t *tci, const double *tv,
                     const double *lo, const double *hi, const double *l, const double *u,
                     const double *c, double sigma, double lambda, int64_t k,
                     const double *x0, const double *y0, double *x, double *y,
                     double *xb, double *yb, double *zb, double *xh, double *work_n, double *work_m) {
    double s = 1.0 / (lambda * sigma);
    double a0 = 1.0 / (double)(k + 2), a1 = (double)(k + 1) / (double)(k + 2);
    /* primal: xbar = Pi_K(x + sigma (A^T y - c)), zbar = (xbar - w) / sigma */
    spmv(n, trp, tci, tv, y, work_n);
    for (int32_t j = 0; j < n; ++j) {
        double w = x[j] + sigma * (work_n[j] - c[j]);
        xb[j] = clampd(w, l[j], u[j]);
        zb[j] = (xb[j] - w) / sigma;
        xh[j] = 2.0 * xb[j] - x[j];
    }
    /* dual: ybar = projection of y - s A(2 xbar - x) */
    spmv(m, rp, ci, v, xh, work_m);
    for (int32_t i = 0; i < m; ++i) {
        double vv = y[i] - s * work_m[i];
        double up = vv + s * lo[i], dn = vv + s * hi[i];
        yb[i] = up > 0.0 ? up : (dn < 0.0 ? dn : 0.0);
    }
    /* reflection and Halpern averaging */
    for (int32_t j = 0; j < n; ++j) x[j] = a0 * x0[j] + a1 * xh[j];
    for (int32_t i = 0; i < m; ++i) {
        double yh = 2.0 * yb[i] - y[i];
        y[i] = a0 * y0[i] + a1 * yh;
    }
}

/* Test entry: one raw step on an unscaled problem. x, y are updated in place. */
int orc_hpr_step(const orc_lp *lp, double sigma, double lambda, int64_t k,
                 const double *x0, const double *y0, double *x, double *y,
                 double *xb, double *yb, double *zb) {
    int32_t m = lp->m, n = lp->n;
    int64_t nnz = lp->nnz;
    int64_t *trp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    double *tv = (double *)malloc(sizeof(double) * ((size_t)nnz + 1));
    int64_t zero = 0;
    const int64_t *rp = m ? lp->row_ptr : &zero;
    transpose(m, n, rp, lp->col_idx, lp->val, trp, tci, tv);
    double *xh = (double *)malloc(sizeof(double) * (size_t)n);
    double *wn = (double *)malloc(sizeof(double) * (size_t)n);
    double *wm = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    hpr_step(m, n, rp, lp->col_idx, lp->val, trp, tci, tv, lp->row_lo, lp->row_hi,
             lp->col_lo, lp->col_hi, lp->c, sigma, lambda, k, x0, y0, x, y, xb, yb, zb, xh, wn, wm);
    free(trp); free(tci); free(tv); free(xh); free(wn); free(wm);
    return 0;
}

/* ---------------------------------------------------------------- the solver */

static void unscale(const scaled_lp *s, const double *xb, const double *yb, const double *zb,
                    double *x, double *y, double *z) {
    for (int32_t j = 0; j < s->n; ++j) {
        x[j] = s->beta_b * s->dc[j] * xb[j];
        z[j] = s->beta_c * zb[j] / s->dc[j];
    }
    for (int32_t i = 0; i < s->m; ++i) y[i] = s->beta_c * s->dr[i] * yb[i];
}

/* Primal infeasibility certificate test (an addition to the method: the paper does not
 * treat infeasible LPs). Weak duality for the row-bounded LP gives, for any feasible x and
 * any y that is sign-feasible (y_i > 0 only where lo_i is finite, y_i < 0 only where hi_i is
 * finite) with dz = -A^T y sign-feasible for the column bounds:
 *     h(y) = sum_i (lo_i y_i+ - hi_i y_i-) + sum_j (l_j dz_j+ - u_j dz_j-)
 *          <= sum_i (Ax)_i y_i + sum_j x_j dz_j = 0,
 * so h(y) > 0 proves that no feasible x exists. Evaluated on the scaled problem at the bar
 * point ybar (sign-feasible by its projection); the ratios below do not change under the
 * diagonal scaling of rows and columns. out: [0] h, [1] sum of the magnitudes of h's terms,
 * [2] sign violations of dz on infinite bounds (zero when every column is bounded), [3] the
 * size of ybar, sum |ybar_i| (the rows of the scaled matrix have norms near 1, so violations
 * are compared with it). aty: n doubles of work. */
static void certificate(const scaled_lp *s, const double *yb, double *aty, double out[4]) {
    double h = 0.0, mag = 0.0, viol = 0.0, ysum = 0.0;
    for (int32_t i = 0; i < s->m; ++i) {
        ysum += fabs(yb[i]);
        if (yb[i] > 0.0) { h += s->lo[i] * yb[i]; mag += fabs(s->lo[i]) * yb[i]; }
        else if (yb[i] < 0.0) { h += s->hi[i] * yb[i]; mag += fabs(s->hi[i]) * -yb[i]; }
    }
    spmv(s->n, s->trp, s->tci, s->tv, yb, aty);   /* A~^T ybar */
    for (int32_t j = 0; j < s->n; ++j) {
        double dz = -aty[j];
        if (dz > 0.0) {
            if (isfinite(s->l[j])) { h += s->l[j] * dz; mag += fabs(s->l[j]) * dz; }
            else viol += dz;
        } else if (dz < 0.0) {
            if (isfinite(s->u[j])) { h += s->u[j] * dz; mag += fabs(s->u[j]) * -dz; }
            else viol += -dz;
        }
    }
    out[0] = h; out[1] = mag; out[2] = viol; out[3] = ysum;
}

static int certifies_infeasibility(const double c[4]) {
    return c[0] > ORC_INFEAS_TOL * c[1] && c[2] <= ORC_INFEAS_TOL * c[3];
}

/* Dual infeasibility (an addition to the method, like the test above). A direction d with
 * c^T d < 0 that the problem's recession cones admit, A d in the rows' cone ((A d)_i = 0 for
 * two finite sides, >= 0 when only lo_i is finite, <= 0 when only hi_i is, free otherwise) and d
 * in the columns' cone (the same rule with l_j, u_j), shows that the dual has no feasible point:
 * the LP has no finite optimum. For such LPs the step's fixed-point residual converges to the
 * operator's minimal displacement, whose primal part is such a ray, so the candidate is the
 * primal move of the step, d = xbar - x (scaled problem; x the iterate the step started from).
 * out: [0] g = c~^T d, [1] ||distance of A~ d to the rows' cone||, [2] ||distance of d to the
 * columns' cone||, [3] ||c~||; work: m doubles. */
static void ray_test(const scaled_lp *s, const double *xb, const double *xprev, double *d, double *ad,
                     double out[4]) {
    double g = 0.0, vr = 0.0, vc = 0.0, c2 = 0.0;
    for (int32_t j = 0; j < s->n; ++j) {
        d[j] = xb[j] - xprev[j];
        g += s->c[j] * d[j];
        c2 += s->c[j] * s->c[j];
        double v = 0.0;
        const int fl = isfinite(s->l[j]), fu = isfinite(s->u[j]);
        if (fl && fu) v = fabs(d[j]);
        else if (fl) v = d[j] < 0.0 ? -d[j] : 0.0;
        else if (fu) v = d[j] > 0.0 ? d[j] : 0.0;
        vc += v * v;
    }
    spmv(s->m, s->rp, s->ci, s->v, d, ad);
    for (int32_t i = 0; i < s->m; ++i) {
        double v = 0.0;
        const int fl = isfinite(s->lo[i]), fh = isfinite(s->hi[i]);
        if (fl && fh) v = fabs(ad[i]);
        else if (fl) v = ad[i] < 0.0 ? -ad[i] : 0.0;
        else if (fh) v = ad[i] > 0.0 ? ad[i] : 0.0;
        vr += v * v;
    }
    out[0] = g; out[1] = sqrt(vr); out[2] = sqrt(vc); out[3] = sqrt(c2);
}

/* d certifies dual infeasibility when it lowers the cost and its cone violations are at most
 * 1e-6 of the cost decrease measured in units of d (-g / ||c~|| <= ||d||). */
static int certifies_unboundedness(const double r[4]) {
    return r[0] < 0.0 && r[3] > 0.0 && r[1] + r[2] <= ORC_INFEAS_TOL * (-r[0] / r[3]);
}

/* ---------------------------------------------------------------- restart and sigma rules */

/*
 * State of the restart rule between checks: r0 is the merit at the last restart (or at the
 * first check), r_prev the merit of the previous check; seen = 0 before the first check.
 */
typedef struct { double r0, r_prev; int64_t seen; } restart_state;

/*
 * Restart decision at one check (the paper names restarts without giving the rule; this is
 * the rule both solvers take). r: the merit of this check; k: steps since the last restart,
 * counting this check's step; done: all steps so far. The first check only records
 * r0 = r_prev = r. Later checks restart when
 *     r <= 0.2 r0   (sufficient decay), or
 *     r <= 0.8 r0 and r > r_prev   (necessary decay without progress), or
 *     k >= 0.2 done   (the current run is a large share of the whole solve);
 * enabled = 0 never restarts. Afterwards r_prev = r, and after a restart r0 = r.
 */
static int restart_decide(restart_state *st, double r, int64_t k, int64_t done, int enabled) {
    if (!st->seen) {
        st->seen = 1;
        st->r0 = r;
        st->r_prev = r;
        return 0;
    }
    int restart = 0;
    if (enabled) {
        if (r <= 0.2 * st->r0) restart = 1;
        else if (r <= 0.8 * st->r0 && r > st->r_prev) restart = 1;
        else if ((double)k >= 0.2 * (double)done) restart = 1;
    }
    if (restart) st->r0 = r;
    st->r_prev = r;
    return restart;
}

/* Test entry: the rule above on a caller-held state [r0, r_prev, seen] (start from zeros). */
int orc_restart_rule(double *state, double r, int64_t k, int64_t done, int32_t enabled) {
    restart_state st = {state[0], state[1], (int64_t)state[2]};
    int d = restart_decide(&st, r, k, done, enabled);
    state[0] = st.r0;
    state[1] = st.r_prev;
    state[2] = (double)st.seen;
    return d;
}

/*
 * sigma at a restart. The bound of Theorem 1 grows with the start's distance in the metric
 * M = [[I/sigma, A^T], [A, lambda sigma I]]; its diagonal part ||dx||^2/sigma + lambda sigma
 * ||dy||^2 is smallest at sigma* = ||dx|| / (sqrt(lambda) ||dy||), with (dx, dy) the move of the
 * anchor. The update follows sigma* in log space with weight w,
 * log sigma <- (1 - w) log sigma + w log sigma* (w = 1 and 1/2 evaluated without exp/log),
 * is skipped when either norm is below 1e-12, and is clamped to [1e-4, 1e4].
 */
static double sigma_next(double sigma, double ndx, double ndy, double lambda, double w) {
    if (!(ndx > 1e-12 && ndy > 1e-12)) return sigma;
    double star = ndx / (sqrt(lambda) * ndy);
    double next = (w == 1.0)   ? star
                  : (w == 0.5) ? sqrt(sigma * star)
                               : exp((1.0 - w) * log(sigma) + w * log(star));
    return clampd(next, 1e-4, 1e4);
}

/* Test entry for the sigma update. */
double orc_sigma_next(double sigma, double ndx, double ndy, double lambda, double w) {
    return sigma_next(sigma, ndx, ndy, lambda, w);
}

/* Fields of one trace record (one check that reached the restart decision). */
enum { TR_IT, TR_K, TR_R, TR_R0, TR_RPREV, TR_RESTART, TR_SIGMA, TR_SIGMA_NEXT, TR_NDX, TR_NDY,
       TR_FIELDS };

/*
 * Full solve. Outputs the unscaled (x, y, z) of the last check and fills info.
 *
 * Schedule: the iteration with global index it (0-based) is a check when
 * it % check_every == 0, and the last allowed iteration is always a check
 * (without a restart decision). At a check:
 *   - KKT of the unscaled (xbar, ybar, zbar); stop if rel_kkt <= tol;
 *   - the primal infeasibility certificate, then the dual infeasibility test of the step's
 *     primal move (stop if either holds);
 *   - merit r = || (x - xbar, y - ybar) ||_M with M = [[I/sigma, A~^T], [A~, lambda sigma I]]
 *     (x, y the iterate the step started from);
 *   - the restart decision of restart_decide with k = steps since the last restart and
 *     done = it + 1;
 *   - on restart: sigma <- sigma_next(sigma, ||xbar - x0||, ||ybar - y0||, lambda, w) (w =
 *     sigma_smoothing from a cold start, sigma_smoothing_warm when a start point is given;
 *     (xbar - x0, ybar - y0) is the move of the anchor), then anchor = current = (xbar, ybar)
 *     and k = 0.
 *
 * Tracing (tests only): when trace != NULL, each check that reaches the restart decision
 * appends TR_FIELDS doubles (iteration index, k, r, r0 and r_prev before the decision, the
 * decision, sigma before and after, the two anchor-move norms; the norms are 0 unless the
 * check restarts with the sigma update on) while fewer than trace_cap records exist;
 * *trace_len receives the count. When vecs != NULL, the check with record index vec_check
 * writes the scaled vectors the decision used: x (the step's start), xbar, x0 (anchor),
 * each n doubles, then y, ybar, y0, each m doubles.
 */
static int solve_impl(const orc_lp *lp, const orc_opts *o, double *x_out, double *y_out, double *z_out,
                      orc_info *info, double *trace, int64_t trace_cap, int64_t *trace_len,
                      int64_t vec_check, double *vecs) {
    memset(info, 0, sizeof(*info));
    if (trace_len) *trace_len = 0;
    if (orc_validate(lp) || o->max_iter < 1 || o->check_every < 1 || !(o->sigma0 > 0)) return -1;
    double t0 = now_s();
    int32_t m = lp->m, n = lp->n;
    scaled_lp s;
    build_scaled(lp, o, &s);
    double lambda = o->lambda_in > 0 ? o->lambda_in : power_lambda(&s, o, NULL);
    double t1 = now_s();

    size_t mm = (size_t)m + 1;
    double *x = (double *)malloc(sizeof(double) * n), *x0 = (double *)malloc(sizeof(double) * n);
    double *xprev = (double *)malloc(sizeof(double) * n);
    double *xb = (double *)malloc(sizeof(double) * n), *zb = (double *)malloc(sizeof(double) * n);
    double *xh = (double *)malloc(sizeof(double) * n), *wn = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * mm), *y0 = (double *)malloc(sizeof(double) * mm);
    double *yprev = (double *)malloc(sizeof(double) * mm);
    double *yb = (double *)malloc(sizeof(double) * mm), *wm = (double *)malloc(sizeof(double) * mm);
    double *dxv = (double *)malloc(sizeof(double) * n), *adx = (double *)malloc(sizeof(double) * mm);
    double *aty = (double *)malloc(sizeof(double) * n), cert[4], ray[4];

    /* start point: projections of the (scaled) warm start, or of zero */
    for (int32_t j = 0; j < n; ++j) {
        double xs = o->x0 ? o->x0[j] / (s.beta_b * s.dc[j]) : 0.0;
        x0[j] = clampd(xs, s.l[j], s.u[j]);
        x[j] = x0[j];
    }
    for (int32_t i = 0; i < m; ++i) {
        double ys = o->y0 ? o->y0[i] / (s.beta_c * s.dr[i]) : 0.0;
        if (!isfinite(s.lo[i]) && ys > 0) ys = 0.0;   /* y_i > 0 needs a finite lower side */
        if (!isfinite(s.hi[i]) && ys < 0) ys = 0.0;   /* y_i < 0 needs a finite upper side */
        y0[i] = ys;
        y[i] = ys;
    }
    double w_sigma = (o->x0 || o->y0) ? o->sigma_smoothing_warm : o->sigma_smoothing;

    double sigma = o->sigma0;
    int64_t k = 0, restarts = 0, it, nrec = 0;
    restart_state rs = {0.0, 0.0, 0};
    double kk[8] = {0};
    int term = ORC_ITER_LIMIT;
    for (it = 0; it < o->max_iter; ++it) {
        memcpy(xprev, x, sizeof(double) * n);
        if (m) memcpy(yprev, y, sizeof(double) * m);
        hpr_step(m, n, s.rp, s.ci, s.v, s.trp, s.tci, s.tv, s.lo, s.hi, s.l, s.u, s.c,
                 sigma, lambda, k, x0, y0, x, y, xb, yb, zb, xh, wn, wm);
        k += 1;
        int last = (it == o->max_iter - 1);
        int timed_out = 0;
        if (!(it % o->check_every == 0 || last)) continue;
        if (o->time_limit > 0 && now_s() - t0 > o->time_limit) timed_out = 1;

        unscale(&s, xb, yb, zb, x_out, y_out, z_out);
        orc_kkt(lp, x_out, y_out, z_out, kk);
        if (isnan(kk[3]) || !isfinite(kk[4])) { term = ORC_NUMERIC_FAIL; break; }
        if (kk[3] <= o->tol) { term = ORC_SOLVED; break; }
        certificate(&s, yb, aty, cert);
        if (certifies_infeasibility(cert)) { term = ORC_PRIMAL_INFEASIBLE; break; }
        ray_test(&s, xb, xprev, dxv, adx, ray);
        if (certifies_unboundedness(ray)) { term = ORC_DUAL_INFEASIBLE; break; }
        if (last) { term = ORC_ITER_LIMIT; break; }
        if (timed_out) { term = ORC_TIME_LIMIT; break; }

        /* merit ||(xprev - xbar, yprev - ybar)||_M */
        for (int32_t j = 0; j < n; ++j) dxv[j] = xprev[j] - xb[j];
        spmv(m, s.rp, s.ci, s.v, dxv, adx);
        double dx2 = dot(n, dxv, dxv), dy2 = 0.0, cross = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            double dy = yprev[i] - yb[i];
            dy2 += dy * dy;
            cross += dy * adx[i];
        }
        double r2 = dx2 / sigma + lambda * sigma * dy2 + 2.0 * cross;
        double r = sqrt(r2 > 0 ? r2 : 0.0);
        if (!isfinite(r)) { term = ORC_NUMERIC_FAIL; break; }

        double *rec = (trace && nrec < trace_cap) ? trace + nrec * TR_FIELDS : NULL;
        if (vecs && nrec == vec_check) {
            memcpy(vecs, xprev, sizeof(double) * n);
            memcpy(vecs + n, xb, sizeof(double) * n);
            memcpy(vecs + 2 * (size_t)n, x0, sizeof(double) * n);
            double *vy = vecs + 3 * (size_t)n;
            if (m) {
                memcpy(vy, yprev, sizeof(double) * m);
                memcpy(vy + m, yb, sizeof(double) * m);
                memcpy(vy + 2 * (size_t)m, y0, sizeof(double) * m);
            }
        }
        if (rec) {
            rec[TR_IT] = (double)it; rec[TR_K] = (double)k; rec[TR_R] = r;
            rec[TR_R0] = rs.r0; rec[TR_RPREV] = rs.r_prev; rec[TR_SIGMA] = sigma;
            rec[TR_NDX] = 0.0; rec[TR_NDY] = 0.0;
        }
        int do_restart = restart_decide(&rs, r, k, it + 1, o->restart);
        if (do_restart) {
            if (o->sigma_update) {
                double ddx = 0.0, ddy = 0.0;
                for (int32_t j = 0; j < n; ++j) { double d = xb[j] - x0[j]; ddx += d * d; }
                for (int32_t i = 0; i < m; ++i) { double d = yb[i] - y0[i]; ddy += d * d; }
                ddx = sqrt(ddx);
                ddy = sqrt(ddy);
                if (rec) { rec[TR_NDX] = ddx; rec[TR_NDY] = ddy; }
                sigma = sigma_next(sigma, ddx, ddy, lambda, w_sigma);
            }
            memcpy(x0, xb, sizeof(double) * n);
            memcpy(x, xb, sizeof(double) * n);
            if (m) { memcpy(y0, yb, sizeof(double) * m); memcpy(y, yb, sizeof(double) * m); }
            k = 0;
            restarts += 1;
        }
        if (rec) { rec[TR_RESTART] = (double)do_restart; rec[TR_SIGMA_NEXT] = sigma; }
        if (trace || vecs) nrec += 1;
    }
    double t2 = now_s();
    if (trace_len) *trace_len = nrec < trace_cap ? nrec : trace_cap;
    info->term = term;
    info->iters = (it < o->max_iter) ? it + 1 : o->max_iter;
    info->restarts = restarts;
    info->rel_p = kk[0]; info->rel_d = kk[1]; info->rel_gap = kk[2]; info->rel_kkt = kk[3];
    info->pobj = kk[4]; info->dobj = kk[5];
    info->lambda = lambda;
    info->sigma = sigma;
    info->setup_s = t1 - t0;
    info->solve_s = t2 - t1;
    free(x); free(x0); free(xprev); free(xb); free(zb); free(xh); free(wn);
    free(y); free(y0); free(yprev); free(yb); free(wm); free(dxv); free(adx); free(aty);
    free_scaled(&s);
    return 0;
}

int orc_solve(const orc_lp *lp, const orc_opts *o, double *x_out, double *y_out, double *z_out,
              orc_info *info) {
    return solve_impl(lp, o, x_out, y_out, z_out, info, NULL, 0, NULL, -1, NULL);
}

/* Test entry: orc_solve with the check trace described at solve_impl. */
int orc_solve_trace(const orc_lp *lp, const orc_opts *o, double *x_out, double *y_out, double *z_out,
                    orc_info *info, double *trace, int64_t trace_cap, int64_t *trace_len,
                    int64_t vec_check, double *vecs) {
    return solve_impl(lp, o, x_out, y_out, z_out, info, trace, trace_cap, trace_len, vec_check, vecs);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the row loops from now on (n >= 1); returns the number now in use */
int orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
