/*
 * CPU ORACLE -- test infrastructure, not part of the product path.
 *
 * The edge loop of flux_oracle.c run on all host cores, as the CPU baseline
 * of the benchmark: the edges are given grouped by a global colouring
 * (Section 2.1: no two edges of one colour increment the same cell), and
 * each colour is one OpenMP parallel loop, so the increments of concurrent
 * iterations never touch the same cell and need no atomics.  The flux is the
 * oracle's own (oracle_lf2d_flux); results equal the sequential loop's up to
 * the order in which each cell's increments are added.
 */
#include <stdint.h>

#include <omp.h>

void oracle_lf2d_flux(const double *xa, const double *xb, const double *qL,
                      const double *qR, double adtL, double adtR, double gm1,
                      double eps, double *f);

/* Threads an OpenMP parallel region of this library uses. */
int32_t oracle_omp_threads(void) { return (int32_t)omp_get_max_threads(); }

/* order[col_off[c] .. col_off[c+1]) lists the edges of colour c. */
void oracle_edge_loop_coloured(int32_t ncol, const int64_t *col_off, const int32_t *order,
                               const int32_t *e2n, const int32_t *e2c, const double *x,
                               const double *q, const double *adt, double gm1, double eps,
                               double *res)
{
    for (int32_t c = 0; c < ncol; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t i = col_off[c]; i < col_off[c + 1]; ++i) {
            const int64_t e = order[i];
            const int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
            const int32_t L = e2c[2 * e], R = e2c[2 * e + 1];
            double f[4];
            oracle_lf2d_flux(x + 2 * (int64_t)a, x + 2 * (int64_t)b, q + 4 * (int64_t)L,
                             q + 4 * (int64_t)R, adt[L], adt[R], gm1, eps, f);
            for (int k = 0; k < 4; ++k) {
                res[4 * (int64_t)L + k] += f[k];
                res[4 * (int64_t)R + k] -= f[k];
            }
        }
    }
}
