/*
 * legacy_omp.c -- the 3D Jacobi sweep of the legacy program as a CPU build
 * runs it: the same loop nest, with its `parallel for` and `reduction(max)`
 * clause handled by OpenMP on the host's cores. This is the comparison the
 * paper makes for every parallel region (the GPU build against the CPU
 * OpenMP build of the same region, Section 5).
 *
 * TIMING ONLY: it is not a parity reference (the serial oracle in oracle.c
 * is) and shares no code with the GPU path. Built with -O2 -fopenmp
 * -ffp-contract=off, so its grids equal the oracle's bit for bit.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

/* Runs `sweeps` sweeps of the n^3 grid on `threads` OpenMP threads (0 = the
 * runtime's default), swapping u and w after each. Returns the max residual
 * of the last sweep. */
double lo_jacobi3d(int64_t n, double *u, double *w, int32_t sweeps, int32_t threads)
{
    const double c6 = 1.0 / 6.0;
    const int64_t sy = n, sz = n * n;
    double *cur = u, *nxt = w;
    double m = -INFINITY;
    if (threads > 0)
        omp_set_num_threads(threads);
    for (int32_t s = 0; s < sweeps; ++s) {
        m = -INFINITY;
#pragma omp parallel for collapse(2) schedule(static) reduction(max : m)
        for (int64_t z = 1; z < n - 1; ++z)
            for (int64_t y = 1; y < n - 1; ++y) {
                const double *c = cur + z * sz + y * sy;
                double *o = nxt + z * sz + y * sy;
                for (int64_t x = 1; x < n - 1; ++x) {
                    const double v = (((c[x - 1] + c[x + 1]) + (c[x - sy] + c[x + sy])) + (c[x - sz] + c[x + sz])) * c6;
                    const double d = fabs(v - c[x]);
                    m = d > m ? d : m;
                    o[x] = v;
                }
            }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    return m;
}

int32_t lo_max_threads(void) { return (int32_t)omp_get_max_threads(); }
