/*
 * oracle.c -- serial CPU reference (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Every function is the legacy loop written out in its natural serial
 * order: the initial thread executing the program alone (paper, Section 2.1).
 * Reductions follow the OpenMP clause semantics the paper leaves to future
 * work (Section 4.3): identity-initialised private copies combined with the
 * original value; here the "combination" is the serial accumulation itself.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Neumaier's improvement of Kahan summation: the running compensation picks
 * up the low-order part lost by each addition, whichever operand is larger. */
static void neumaier_add(double *sum, double *comp, double t)
{
    double s = *sum + t;
    if (fabs(*sum) >= fabs(t))
        *comp += (*sum - s) + t;
    else
        *comp += (t - s) + *sum;
    *sum = s;
}

/* ------------------------------------------------------------------------ */
/* 2D 5-point Jacobi (the 2D legacy-loop program)                           */
/* ------------------------------------------------------------------------ */

static int64_t append_line(char *text, int64_t cap, int64_t used, int32_t sweep, double res)
{
    if (!text || cap <= 0)
        return used;
    if (used >= cap - 1)
        return used;
    int k = snprintf(text + used, (size_t)(cap - used), "sweep %d residual %.10e\n", sweep, res);
    if (k < 0)
        return used;
    used += k;
    if (used > cap - 1)
        used = cap - 1;
    return used;
}

int or_jacobi2d(int64_t n, double *u, double *w, int32_t sweeps, double *res,
                double *res_comp, int32_t print_every, char *text, int64_t text_cap)
{
    double *cur = u, *nxt = w;
    int64_t used = 0;
    if (text && text_cap > 0)
        text[0] = '\0';
    for (int32_t s = 1; s <= sweeps; ++s) {
        double acc = 0.0, cs = 0.0, cc = 0.0;
        for (int64_t j = 1; j < n - 1; ++j) {
            for (int64_t i = 1; i < n - 1; ++i) {
                const double *c = cur + j * n + i;
                double v = ((c[-1] + c[1]) + (c[-n] + c[n])) * 0.25;
                double d = v - c[0];
                acc = acc + d * d;
                neumaier_add(&cs, &cc, d * d);
                nxt[j * n + i] = v;
            }
        }
        double r = sqrt(acc);
        if (res)
            res[s - 1] = r;
        if (res_comp)
            res_comp[s - 1] = sqrt(cs + cc);
        double *t = cur;
        cur = nxt;
        nxt = t;
        if (print_every > 0 && s % print_every == 0)
            used = append_line(text, text_cap, used, s, r);
    }
    return cur == u ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* 3D 7-point Jacobi (the 3D legacy-loop program)                           */
/* ------------------------------------------------------------------------ */

int or_jacobi3d(int64_t n, double *u, double *w, int32_t sweeps, double *res)
{
    const double c6 = 1.0 / 6.0;
    const int64_t sy = n, sz = n * n;
    double *cur = u, *nxt = w;
    for (int32_t s = 1; s <= sweeps; ++s) {
        double m = -INFINITY;
        for (int64_t z = 1; z < n - 1; ++z) {
            for (int64_t y = 1; y < n - 1; ++y) {
                for (int64_t x = 1; x < n - 1; ++x) {
                    const double *c = cur + z * sz + y * sy + x;
                    double v = (((c[-1] + c[1]) + (c[-sy] + c[sy])) + (c[-sz] + c[sz])) * c6;
                    double d = fabs(v - c[0]);
                    if (d > m)
                        m = d;
                    nxt[z * sz + y * sy + x] = v;
                }
            }
        }
        if (res)
            res[s - 1] = m;
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    return cur == u ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* CG building blocks                                                       */
/* ------------------------------------------------------------------------ */

void or_spmv_csr(int64_t nrows, const int32_t *rowptr, const int32_t *col,
                 const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double acc = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            acc = acc + val[k] * x[col[k]];
        y[i] = acc;
    }
}

double or_dot(int64_t n, const double *a, const double *b)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        acc = acc + a[i] * b[i];
    return acc;
}

double or_dot_compensated(int64_t n, const double *a, const double *b, double *abs_sum)
{
    double s = 0.0, c = 0.0, as = 0.0, ac = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = a[i] * b[i];
        neumaier_add(&s, &c, t);
        neumaier_add(&as, &ac, fabs(t));
    }
    if (abs_sum)
        *abs_sum = as + ac;
    return s + c;
}

void or_axpby(int64_t n, double *out, const double *x, double s, const double *y)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = x[i] + s * y[i];
}

int32_t or_cg_iteration(int64_t nrows, const int32_t *rowptr, const int32_t *col,
                        const double *val, double *x, double *r, double *p, double *q,
                        double *rho, double *pq_out, double *alpha_out, double *beta_out)
{
    or_spmv_csr(nrows, rowptr, col, val, p, q);
    double pq = or_dot(nrows, p, q);
    if (pq_out)
        *pq_out = pq;
    if (pq == 0.0 || *rho == 0.0)
        return 1;
    double alpha = *rho / pq;
    for (int64_t i = 0; i < nrows; ++i)
        x[i] = x[i] + alpha * p[i];
    for (int64_t i = 0; i < nrows; ++i)
        r[i] = r[i] - alpha * q[i];
    double rho_new = or_dot(nrows, r, r);
    double beta = rho_new / *rho;
    *rho = rho_new;
    for (int64_t i = 0; i < nrows; ++i)
        p[i] = r[i] + beta * p[i];
    if (alpha_out)
        *alpha_out = alpha;
    if (beta_out)
        *beta_out = beta;
    return 0;
}

int32_t or_cg(int64_t nrows, const int32_t *rowptr, const int32_t *col, const double *val,
              const double *b, double *x, int32_t iters, double *rho_hist,
              double *alpha_hist, double *beta_hist, int32_t compensated)
{
    double *r = (double *)malloc((size_t)nrows * sizeof(double));
    double *p = (double *)malloc((size_t)nrows * sizeof(double));
    double *q = (double *)malloc((size_t)nrows * sizeof(double));
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        return -1;
    }
    for (int64_t i = 0; i < nrows; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        p[i] = r[i];
    }
    double rho = compensated ? or_dot_compensated(nrows, r, r, NULL) : or_dot(nrows, r, r);
    int32_t k = 0;
    for (; k < iters; ++k) {
        if (rho == 0.0)
            break;
        or_spmv_csr(nrows, rowptr, col, val, p, q);
        double pq = compensated ? or_dot_compensated(nrows, p, q, NULL) : or_dot(nrows, p, q);
        if (pq == 0.0)
            break;
        double alpha = rho / pq;
        for (int64_t i = 0; i < nrows; ++i)
            x[i] = x[i] + alpha * p[i];
        for (int64_t i = 0; i < nrows; ++i)
            r[i] = r[i] - alpha * q[i];
        double rho_new = compensated ? or_dot_compensated(nrows, r, r, NULL) : or_dot(nrows, r, r);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < nrows; ++i)
            p[i] = r[i] + beta * p[i];
        if (rho_hist)
            rho_hist[k] = rho;
        if (alpha_hist)
            alpha_hist[k] = alpha;
        if (beta_hist)
            beta_hist[k] = beta;
    }
    free(r);
    free(p);
    free(q);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Histogram and reductions                                                 */
/* ------------------------------------------------------------------------ */

void or_hist_u32(int64_t n, const uint32_t *keys, uint32_t *bins, uint32_t mask)
{
    for (int64_t t = 0; t < n; ++t)
        bins[keys[t] & mask] += 1u;
}

double or_sum_f64(int64_t n, const double *x)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        acc = acc + x[i];
    return acc;
}

double or_sum_f64_compensated(int64_t n, const double *x)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i)
        neumaier_add(&s, &c, x[i]);
    return s + c;
}

double or_max_f64(int64_t n, const double *x)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (x[i] > m)
            m = x[i];
    return m;
}

uint64_t or_sum_u32(int64_t n, const uint32_t *x)
{
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; ++i)
        acc += x[i];
    return acc;
}

uint64_t or_sum_u64(int64_t n, const uint64_t *x)
{
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; ++i)
        acc += x[i];
    return acc;
}

int64_t or_sum_i64(int64_t n, const int64_t *x)
{
    uint64_t acc = 0; /* two's-complement wrap without signed overflow */
    for (int64_t i = 0; i < n; ++i)
        acc += (uint64_t)x[i];
    return (int64_t)acc;
}

uint32_t or_max_u32(int64_t n, const uint32_t *x)
{
    uint32_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (x[i] > m)
            m = x[i];
    return m;
}

uint64_t or_max_u64(int64_t n, const uint64_t *x)
{
    uint64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (x[i] > m)
            m = x[i];
    return m;
}

int64_t or_max_i64(int64_t n, const int64_t *x)
{
    int64_t m = INT64_MIN;
    for (int64_t i = 0; i < n; ++i)
        if (x[i] > m)
            m = x[i];
    return m;
}

/* ------------------------------------------------------------------------ */
/* Static worksharing                                                       */
/* ------------------------------------------------------------------------ */

void or_static_owner(int64_t n, int64_t nthreads, int64_t chunk, int32_t *owner)
{
    if (nthreads <= 0)
        return;
    if (chunk > 0) {
        for (int64_t i = 0; i < n; ++i)
            owner[i] = (int32_t)((i / chunk) % nthreads);
        return;
    }
    int64_t q = n / nthreads, r = n % nthreads;
    for (int64_t t = 0; t < nthreads; ++t) {
        int64_t lo = t * q + (t < r ? t : r);
        int64_t hi = (t + 1) * q + (t + 1 < r ? t + 1 : r);
        for (int64_t i = lo; i < hi; ++i)
            owner[i] = (int32_t)t;
    }
}

/* Producer/consumer phases of a `parallel` region with manual worksharing
 * and barriers (Section 3.3). Every phase p computes dst[i] = src[i] +
 * src[(i + shift) % n] for all i and then swaps the roles of the two
 * arrays. Which thread computes which i, and the barrier that separates the
 * phases, do not change the values, so the serial program is these loops in
 * index order. The result ends in a after an even number of phases and in
 * b after an odd one. */
void or_phases(int64_t n, double *a, double *b, int64_t phases, int64_t shift)
{
    double *src = a, *dst = b;
    for (int64_t p = 0; p < phases; ++p) {
        for (int64_t i = 0; i < n; ++i)
            dst[i] = src[i] + src[(i + shift) % n];
        double *t = src;
        src = dst;
        dst = t;
    }
}
