/*
 * FP64 CPU oracle for cubic-spline interpolation (Hornbeck, "Fast Cubic
 * Spline Interpolation", arXiv 2001.09253).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the HIP
 * library.
 *
 * The oracle computes the plain definitions the method reaches exactly:
 *
 *   1. the tridiagonal system whose rows are the first-derivative continuity
 *      condition of the section "Generating Second Derivatives" (equation
 *      eqn:init_val and the a_j, b_j, c_j, d_j that follow it), with the end
 *      rows of the section "Start and End Derivatives";
 *   2. the solution of that system by Gaussian elimination with partial
 *      pivoting on the band (a textbook routine, deliberately not Thomas'
 *      algorithm, so that the oracle does not follow the paper's solver);
 *   3. the interval of each query found by binary search;
 *   4. the interpolant in the A, B, C, D form of equation eqn:nr_formula
 *      (section "Fast Interpolation"), not the rewritten form the paper
 *      derives from it.
 *
 * Readings of the paper taken here (they are the ones the HIP path takes):
 *   - an end is natural iff its derivative argument is > 0.99e30 (the
 *     sentinel of the paper's routine); otherwise it is clamped to that slope;
 *   - the clamped end rows are
 *       start: 2h y''_0 + h y''_1 = 6((y_1 - y_0)/h - y'_start)
 *       end:   h y''_{n-2} + 2h y''_{n-1} = 6(y'_end - (y_{n-1} - y_{n-2})/h)
 *     (the end row follows the derived equation, whose coefficient order the
 *     prose after it swaps);
 *   - a natural end row is y''_end = 0;
 *   - knots must be strictly increasing and n >= 3;
 *   - query k of m uniform queries is x_0 + k*h with h = (x_{n-1}-x_0)/(m-1),
 *     one multiply then one add (no fused multiply-add), and the last query
 *     is x_{n-1} itself;
 *   - the interval of query q is clip(#{j : x_j < q} - 1, 0, n-2), which is
 *     the interval the paper's bracketing loop stops at for queries inside
 *     [x_0, x_{n-1}]; queries outside use the end intervals.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_SIZE (-2)
#define ORACLE_E_ORDER (-3)
#define ORACLE_E_SINGULAR (-8)
#define ORACLE_E_NOMEM (-9)

/* Natural-end sentinel of the paper's second-derivative routine. */
static int oracle_is_natural(double deriv) { return deriv > 0.99e30; }

/* Preconditions asserted by the paper's routines: n > 2 and strictly
 * increasing knots.  A NaN knot fails the strict comparison. */
int oracle_validate(const double *x, int64_t n)
{
    if (n < 3) return ORACLE_E_SIZE;
    if (!x) return ORACLE_E_ARG;
    for (int64_t j = 1; j < n; ++j)
        if (!(x[j] > x[j - 1])) return ORACLE_E_ORDER;
    return ORACLE_OK;
}

/*
 * Rows of T y'' = d.  Row j reads  lo[j] y''_{j-1} + di[j] y''_j + up[j] y''_{j+1} = rhs[j].
 * Interior rows (1 <= j <= n-2), section "Generating Second Derivatives":
 *   lo = x_j - x_{j-1},  di = 2 (x_{j+1} - x_{j-1}),  up = x_{j+1} - x_j,
 *   rhs = 6 ((y_{j+1} - y_j)/(x_{j+1} - x_j) - (y_j - y_{j-1})/(x_j - x_{j-1})).
 * End rows, section "Start and End Derivatives" (see the header comment).
 */
int oracle_rows(const double *x, const double *y, int64_t n, double start_deriv,
                double end_deriv, double *lo, double *di, double *up, double *rhs)
{
    int rc = oracle_validate(x, n);
    if (rc) return rc;
    if (!y || !lo || !di || !up || !rhs) return ORACLE_E_ARG;
    for (int64_t j = 1; j + 1 < n; ++j) {
        lo[j] = x[j] - x[j - 1];
        di[j] = 2.0 * (x[j + 1] - x[j - 1]);
        up[j] = x[j + 1] - x[j];
        rhs[j] = 6.0 * ((y[j + 1] - y[j]) / (x[j + 1] - x[j]) - (y[j] - y[j - 1]) / (x[j] - x[j - 1]));
    }
    lo[0] = 0.0;
    if (oracle_is_natural(start_deriv)) {
        di[0] = 1.0;
        up[0] = 0.0;
        rhs[0] = 0.0;
    } else {
        double h = x[1] - x[0];
        di[0] = 2.0 * h;
        up[0] = h;
        rhs[0] = 6.0 * ((y[1] - y[0]) / h - start_deriv);
    }
    up[n - 1] = 0.0;
    if (oracle_is_natural(end_deriv)) {
        lo[n - 1] = 0.0;
        di[n - 1] = 1.0;
        rhs[n - 1] = 0.0;
    } else {
        double h = x[n - 1] - x[n - 2];
        lo[n - 1] = h;
        di[n - 1] = 2.0 * h;
        rhs[n - 1] = 6.0 * (end_deriv - (y[n - 1] - y[n - 2]) / h);
    }
    return ORACLE_OK;
}

/*
 * Gaussian elimination with partial pivoting on a tridiagonal band, then back
 * substitution.  Pivoting may move a row up by one, which fills a second
 * super-diagonal (f2).  Inputs are copied; out[n] receives the solution.
 */
int oracle_band_solve(int64_t n, const double *lo_in, const double *di_in,
                      const double *up_in, const double *rhs_in, double *out)
{
    if (n < 1 || !lo_in || !di_in || !up_in || !rhs_in || !out) return ORACLE_E_ARG;
    double *sub = (double *)malloc(sizeof(double) * (size_t)n);   /* sub[k]: entry (k+1, k) */
    double *dg = (double *)malloc(sizeof(double) * (size_t)n);
    double *f1 = (double *)malloc(sizeof(double) * (size_t)n);    /* entry (k, k+1) */
    double *f2 = (double *)malloc(sizeof(double) * (size_t)n);    /* entry (k, k+2) */
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = ORACLE_OK;
    if (!sub || !dg || !f1 || !f2 || !r) { rc = ORACLE_E_NOMEM; goto done; }
    for (int64_t k = 0; k < n; ++k) {
        sub[k] = (k + 1 < n) ? lo_in[k + 1] : 0.0;
        dg[k] = di_in[k];
        f1[k] = up_in[k];
        f2[k] = 0.0;
        r[k] = rhs_in[k];
    }
    for (int64_t k = 0; k + 1 < n; ++k) {
        if (fabs(dg[k]) >= fabs(sub[k])) {
            /* pivot stays on row k */
            if (dg[k] == 0.0) { rc = ORACLE_E_SINGULAR; goto done; }
            double l = sub[k] / dg[k];
            dg[k + 1] -= l * f1[k];
            r[k + 1] -= l * r[k];
            /* f2[k] is still zero here, so row k+1's column k+2 is unchanged */
        } else {
            /* swap rows k and k+1, then eliminate */
            double l = dg[k] / sub[k];
            double row1_d = sub[k], row1_f1 = dg[k + 1], row1_f2 = (k + 2 < n) ? f1[k + 1] : 0.0;
            double row2_f0 = f1[k];             /* old row k, column k+1 */
            double r1 = r[k + 1], r2 = r[k];
            dg[k] = row1_d;
            f1[k] = row1_f1;
            f2[k] = row1_f2;
            /* new row k+1 = old row k - l * new row k */
            dg[k + 1] = row2_f0 - l * row1_f1;
            if (k + 2 < n) f1[k + 1] = 0.0 - l * row1_f2;
            r[k] = r1;
            r[k + 1] = r2 - l * r1;
        }
    }
    if (dg[n - 1] == 0.0) { rc = ORACLE_E_SINGULAR; goto done; }
    out[n - 1] = r[n - 1] / dg[n - 1];
    if (n >= 2) out[n - 2] = (r[n - 2] - f1[n - 2] * out[n - 1]) / dg[n - 2];
    for (int64_t k = n - 3; k >= 0; --k)
        out[k] = (r[k] - f1[k] * out[k + 1] - f2[k] * out[k + 2]) / dg[k];
done:
    free(sub); free(dg); free(f1); free(f2); free(r);
    return rc;
}

/* Second derivatives at the knots: assemble the rows, then solve them. */
int oracle_second_derivatives(const double *x, const double *y, int64_t n,
                              double start_deriv, double end_deriv, double *ypp)
{
    int rc = oracle_validate(x, n);
    if (rc) return rc;
    if (!y || !ypp) return ORACLE_E_ARG;
    double *buf = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    if (!buf) return ORACLE_E_NOMEM;
    double *lo = buf, *di = buf + n, *up = buf + 2 * n, *rhs = buf + 3 * n;
    rc = oracle_rows(x, y, n, start_deriv, end_deriv, lo, di, up, rhs);
    if (!rc) rc = oracle_band_solve(n, lo, di, up, rhs, ypp);
    free(buf);
    return rc;
}

/* Query k of m uniform queries between x_0 and x_last (reading A5). */
double oracle_uniform_query(double x0, double xlast, int64_t m, int64_t k)
{
    if (m <= 1 || k <= 0) return x0;
    if (k >= m - 1) return xlast;
    double h = (xlast - x0) / (double)(m - 1);
    double step = (double)k * h;
    return x0 + step;
}

void oracle_uniform_queries(double x0, double xlast, int64_t m, double *q)
{
    for (int64_t k = 0; k < m; ++k) q[k] = oracle_uniform_query(x0, xlast, m, k);
}

/* Interval of query q: clip(#{j : x_j < q} - 1, 0, n-2), by binary search. */
int64_t oracle_bracket(const double *x, int64_t n, double q)
{
    int64_t lo = 0, hi = n;            /* answer cnt in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (x[mid] < q) lo = mid + 1; else hi = mid;
    }
    int64_t i = lo - 1;
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    return i;
}

/* The interpolant on interval i in the A, B, C, D form (eqn:nr_formula). */
double oracle_eval_interval(const double *x, const double *y, const double *ypp,
                            int64_t i, double q)
{
    double h = x[i + 1] - x[i];
    double A = (x[i + 1] - q) / h;
    double B = (q - x[i]) / h;
    double C = (A * A * A - A) * (h * h) / 6.0;
    double D = (B * B * B - B) * (h * h) / 6.0;
    return A * y[i] + B * y[i + 1] + C * ypp[i] + D * ypp[i + 1];
}

/* First and second derivative of the interpolant on interval i, obtained by
 * differentiating the A, B, C, D form with dA/dx = -1/h, dB/dx = 1/h. */
void oracle_eval_derivs(const double *x, const double *y, const double *ypp,
                        int64_t i, double q, double *d1, double *d2)
{
    double h = x[i + 1] - x[i];
    double A = (x[i + 1] - q) / h;
    double B = (q - x[i]) / h;
    *d1 = (y[i + 1] - y[i]) / h - (3.0 * A * A - 1.0) * h / 6.0 * ypp[i]
          + (3.0 * B * B - 1.0) * h / 6.0 * ypp[i + 1];
    *d2 = A * ypp[i] + B * ypp[i + 1];
}

/* Evaluate at explicit queries; idx (nullable) receives the intervals. */
int oracle_eval_points(const double *x, const double *y, const double *ypp, int64_t n,
                       const double *q, int64_t m, double *yq, int64_t *idx)
{
    if (n < 2 || m < 0 || !x || !y || !ypp || (m && (!q || !yq))) return ORACLE_E_ARG;
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = oracle_bracket(x, n, q[k]);
        if (idx) idx[k] = i;
        yq[k] = oracle_eval_interval(x, y, ypp, i, q[k]);
    }
    return ORACLE_OK;
}

/* Derivatives at explicit queries (either output may be NULL). */
int oracle_eval_points_derivs(const double *x, const double *y, const double *ypp, int64_t n,
                              const double *q, int64_t m, double *d1, double *d2)
{
    if (n < 2 || m < 0 || !x || !y || !ypp || (m && !q)) return ORACLE_E_ARG;
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = oracle_bracket(x, n, q[k]);
        double a, b;
        oracle_eval_derivs(x, y, ypp, i, q[k], &a, &b);
        if (d1) d1[k] = a;
        if (d2) d2[k] = b;
    }
    return ORACLE_OK;
}

/* Intervals of the m uniform queries. */
int oracle_bracket_uniform(const double *x, int64_t n, int64_t m, int64_t *idx)
{
    if (n < 2 || m < 1 || !x || !idx) return ORACLE_E_ARG;
    for (int64_t k = 0; k < m; ++k)
        idx[k] = oracle_bracket(x, n, oracle_uniform_query(x[0], x[n - 1], m, k));
    return ORACLE_OK;
}

/* Whole path for one instance: second derivatives, then m uniform queries. */
int oracle_spline_uniform(const double *x, const double *y, int64_t n, double start_deriv,
                          double end_deriv, int64_t m, double *yq, double *ypp_out)
{
    if (m < 1) return ORACLE_E_SIZE;
    int rc = oracle_validate(x, n);
    if (rc) return rc;
    if (!y || !yq) return ORACLE_E_ARG;
    double *ypp = ypp_out ? ypp_out : (double *)malloc(sizeof(double) * (size_t)n);
    if (!ypp) return ORACLE_E_NOMEM;
    rc = oracle_second_derivatives(x, y, n, start_deriv, end_deriv, ypp);
    if (!rc) {
        for (int64_t k = 0; k < m; ++k) {
            double q = oracle_uniform_query(x[0], x[n - 1], m, k);
            yq[k] = oracle_eval_interval(x, y, ypp, oracle_bracket(x, n, q), q);
        }
    }
    if (!ypp_out) free(ypp);
    return rc;
}

/*
 * Uniform queries k0 .. k1-1 of m (reading A5) on a curve whose second
 * derivatives ypp are given: yq[k - k0] is the value at query k and, when idx
 * is not NULL, idx[k - k0] its interval.  Each query is positioned, bracketed
 * and evaluated on its own exactly as in oracle_spline_uniform; the queries
 * are spread over `threads` OpenMP threads (<= 0: the OpenMP default), which
 * changes no arithmetic.  Lets a caller check a long run of queries chunk by
 * chunk.
 */
int oracle_uniform_range(const double *x, const double *y, const double *ypp, int64_t n, int64_t m,
                         int64_t k0, int64_t k1, double *yq, int64_t *idx, int threads)
{
    if (n < 2 || m < 1 || k0 < 0 || k1 > m || k0 > k1 || !x || !y || !ypp || !yq) return ORACLE_E_ARG;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
#else
    (void)threads;
#endif
    for (int64_t k = k0; k < k1; ++k) {
        double q = oracle_uniform_query(x[0], x[n - 1], m, k);
        int64_t i = oracle_bracket(x, n, q);
        if (idx) idx[k - k0] = i;
        yq[k - k0] = oracle_eval_interval(x, y, ypp, i, q);
    }
    return ORACLE_OK;
}

/* Only a sample of the uniform queries: yq[r] = value at query index ks[r]. */
int oracle_spline_uniform_sample(const double *x, const double *y, int64_t n, double start_deriv,
                                 double end_deriv, int64_t m, const int64_t *ks, int64_t count,
                                 double *yq, double *ypp_out)
{
    if (m < 1) return ORACLE_E_SIZE;
    int rc = oracle_validate(x, n);
    if (rc) return rc;
    double *ypp = ypp_out ? ypp_out : (double *)malloc(sizeof(double) * (size_t)n);
    if (!ypp) return ORACLE_E_NOMEM;
    rc = oracle_second_derivatives(x, y, n, start_deriv, end_deriv, ypp);
    if (!rc) {
        for (int64_t r = 0; r < count; ++r) {
            double q = oracle_uniform_query(x[0], x[n - 1], m, ks[r]);
            yq[r] = oracle_eval_interval(x, y, ypp, oracle_bracket(x, n, q), q);
        }
    }
    if (!ypp_out) free(ypp);
    return rc;
}

/*
 * Many instances in CSR form (instance i: knots koff[i]..koff[i+1], queries
 * qoff[i]..qoff[i+1]); instances are spread over `threads` OpenMP threads
 * (<= 0: the OpenMP default).  status[i] receives each instance's code.
 * Returns the number of threads used.
 */
int oracle_batch_uniform(int64_t count, const int64_t *koff, const int64_t *qoff,
                         const double *x, const double *y, const double *sd, const double *ed,
                         double *yq, double *ypp, int32_t *status, int threads)
{
    int used = 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i) {
            int rc = oracle_spline_uniform(x + koff[i], y + koff[i], koff[i + 1] - koff[i], sd[i], ed[i],
                                           qoff[i + 1] - qoff[i], yq + qoff[i], ypp ? ypp + koff[i] : NULL);
            if (status) status[i] = rc;
        }
    }
#else
    (void)threads;
    for (int64_t i = 0; i < count; ++i) {
        int rc = oracle_spline_uniform(x + koff[i], y + koff[i], koff[i + 1] - koff[i], sd[i], ed[i],
                                       qoff[i + 1] - qoff[i], yq + qoff[i], ypp ? ypp + koff[i] : NULL);
        if (status) status[i] = rc;
    }
#endif
    return used;
}

/* Monotonic wall clock in seconds (for the CPU-baseline timing). */
double oracle_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}
