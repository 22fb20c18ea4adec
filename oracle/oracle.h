/*
 * oracle.h -- serial CPU reference for the GPU-First legacy-loop hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * What it computes is the plain definition of the legacy program: one
 * initial thread runs the serial code and every `parallel for` loop in
 * iteration order (paper, Section 2.1 "OpenMP Execution Model"), with the
 * multi-team rewrite of Section 3.3 changing only *who* executes an
 * iteration, never *what* it computes. The paper leaves reduction clauses
 * unrewritten (Section 4.3), so reductions follow OpenMP semantics: the
 * private copies start at the operator identity and the result is the
 * original value combined with every contribution, in an unspecified order.
 *
 * Build: gcc -O2 -ffp-contract=off -std=c11 (no contraction into FMA, IEEE
 * division and sqrt), so every elementwise value is exactly rounded in the
 * order written.
 */
#ifndef GF_ORACLE_H
#define GF_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- stencil programs ------------------------------------------------- */

/* 2D 5-point Jacobi on an n x n row-major grid with a fixed zero boundary.
 * Each sweep: v = ((W + E) + (S + N)) * 0.25 for every interior point in
 * row-major order, d = v - u, acc += d*d, then res = sqrt(acc), swap, and
 * every `print_every` sweeps (if > 0) one line "sweep %d residual %.10e\n"
 * is appended to `text` (capacity text_cap, always NUL-terminated).
 * u and w both hold the boundary. Returns 0 if the final grid is in u,
 * 1 if it is in w. res[s-1] receives the residual of sweep s (serial sum);
 * res_comp (nullable) the same with a Neumaier-compensated sum. */
int or_jacobi2d(int64_t n, double *u, double *w, int32_t sweeps, double *res,
                double *res_comp, int32_t print_every, char *text, int64_t text_cap);

/* 3D 7-point Jacobi on u[z][y][x] (x fastest), n^3, zero boundary:
 * v = (((xm + xp) + (ym + yp)) + (zm + zp)) * (1.0/6.0), d = v - u,
 * res = max |d| over the sweep (starting from -infinity). Returns 0/1 as
 * or_jacobi2d. */
int or_jacobi3d(int64_t n, double *u, double *w, int32_t sweeps, double *res);

/* ---- CG building blocks ------------------------------------------------ */

/* y = A x for CSR A; each row is summed serially in stored column order. */
void or_spmv_csr(int64_t nrows, const int32_t *rowptr, const int32_t *col,
                 const double *val, const double *x, double *y);
/* Plain serial dot product in index order (the legacy loop's value). */
double or_dot(int64_t n, const double *a, const double *b);
/* Neumaier-compensated dot product; *abs_sum (nullable) receives sum |a_i b_i|. */
double or_dot_compensated(int64_t n, const double *a, const double *b, double *abs_sum);
/* out[i] = x[i] + s * y[i] (out may alias x or y). */
void or_axpby(int64_t n, double *out, const double *x, double s, const double *y);
/* Conjugate gradients with each step a separate loop: q = A p; pq = p.q;
 * alpha = rho/pq; x += alpha p; r -= alpha q; rho' = r.r; beta = rho'/rho;
 * p = r + beta p. x0 = 0. rho_hist[k-1] = rho after iteration k.
 * alpha_hist/beta_hist (nullable) likewise. compensated != 0 uses the
 * compensated dot. Returns the number of iterations completed (stops early
 * on pq == 0 or rho == 0). */
int32_t or_cg(int64_t nrows, const int32_t *rowptr, const int32_t *col, const double *val,
              const double *b, double *x, int32_t iters, double *rho_hist,
              double *alpha_hist, double *beta_hist, int32_t compensated);
/* One CG iteration from state (x, r, p, rho); updates them in place and
 * writes q (scratch of length nrows) and the iteration's pq, alpha, beta.
 * Returns 1 on a breakdown (pq == 0 or rho == 0), else 0. */
int32_t or_cg_iteration(int64_t nrows, const int32_t *rowptr, const int32_t *col,
                        const double *val, double *x, double *r, double *p, double *q,
                        double *rho, double *pq_out, double *alpha_out, double *beta_out);

/* ---- histogram and plain reductions ------------------------------------ */

/* bins[key & mask] += 1 for every key, in order. bins are not cleared. */
void or_hist_u32(int64_t n, const uint32_t *keys, uint32_t *bins, uint32_t mask);

double or_sum_f64(int64_t n, const double *x);              /* serial, index order */
double or_sum_f64_compensated(int64_t n, const double *x);  /* Neumaier */
double or_max_f64(int64_t n, const double *x);              /* from -infinity */
uint64_t or_sum_u32(int64_t n, const uint32_t *x);          /* widened, exact */
uint64_t or_sum_u64(int64_t n, const uint64_t *x);          /* mod 2^64 */
int64_t or_sum_i64(int64_t n, const int64_t *x);            /* mod 2^64 */
uint32_t or_max_u32(int64_t n, const uint32_t *x);
uint64_t or_max_u64(int64_t n, const uint64_t *x);
int64_t or_max_i64(int64_t n, const int64_t *x);

/* ---- worksharing --------------------------------------------------------- */

/* Owner thread of each iteration of a static schedule over T threads with
 * continuous global ids (Section 3.3): chunk == 0 splits [0, n) into T
 * contiguous blocks whose sizes differ by at most one (the first n % T get
 * one more); chunk > 0 deals chunks of that size round-robin. */
void or_static_owner(int64_t n, int64_t nthreads, int64_t chunk, int32_t *owner);
void or_phases(int64_t n, double *a, double *b, int64_t phases, int64_t shift);

#ifdef __cplusplus
}
#endif
#endif
