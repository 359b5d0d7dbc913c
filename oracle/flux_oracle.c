/*
 * CPU ORACLE -- test infrastructure, not part of the product path.
 *
 * Plain sequential binary64 implementation of the indirect-increment edge
 * loop the GPU library accelerates.  Only the tests, the smoke check and the
 * CPU baseline leg of the benchmark may load it.  It shares no code with the
 * HIP library: no headers, helpers or constants.
 *
 * Built with -O2 -ffp-contract=off: every + - * / is one correctly rounded
 * binary64 operation in the order written below.
 *
 * What is computed (paper, Section 1.1.1 "Unstructured meshes" and the
 * Airfoil res_calc description in Section 3.1.1): a loop over the interior
 * edges that reads 2 node coordinates through edge->node, 4 conserved
 * variables and 1 time-step scalar on each of 2 cells through edge->cell,
 * evaluates a flux of about 100 flops, and increments 4 residual values on
 * both cells.  The paper fixes this data volume but prints no formula, so
 * the flux is our own: a central Euler flux with scalar Lax-Friedrichs
 * (Rusanov-type) dissipation,
 *
 *   n    = (y_b - y_a, x_a - x_b)                 (points from L into R)
 *   per side s in {L, R}:
 *     ri = 1 / q0;  u = q1 ri;  v = q2 ri
 *     p  = gm1 (q3 - 0.5 (q1 u + q2 v))
 *     U  = u n_x + v n_y
 *     F  = (q0 U, q1 U + p n_x, q2 U + p n_y, (q3 + p) U)
 *   mu   = eps 0.5 (adt_L + adt_R)
 *   f_k  = 0.5 (F_L,k + F_R,k) + 0.5 mu (q_L,k - q_R,k)
 *   res[L] += f,  res[R] -= f.
 *
 * The loop order is the edge order given (Section 1.1.1: the result must not
 * depend on the processing order beyond rounding).
 */
#include <stdint.h>
#include <string.h>

static void oracle_side_flux(const double *q, double nx, double ny, double gm1,
                             double F[4])
{
    double ri = 1.0 / q[0];
    double u = q[1] * ri;
    double v = q[2] * ri;
    double p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    double U = u * nx + v * ny;
    F[0] = q[0] * U;
    F[1] = q[1] * U + p * nx;
    F[2] = q[2] * U + p * ny;
    F[3] = (q[3] + p) * U;
}

/* Flux through one edge from cell L into cell R. */
void oracle_lf2d_flux(const double *xa, const double *xb, const double *qL,
                      const double *qR, double adtL, double adtR, double gm1,
                      double eps, double *f)
{
    double nx = xb[1] - xa[1];
    double ny = xa[0] - xb[0];
    double FL[4], FR[4];
    oracle_side_flux(qL, nx, ny, gm1, FL);
    oracle_side_flux(qR, nx, ny, gm1, FR);
    double mu = eps * 0.5 * (adtL + adtR);
    for (int k = 0; k < 4; ++k)
        f[k] = 0.5 * (FL[k] + FR[k]) + 0.5 * mu * (qL[k] - qR[k]);
}

/*
 * Sequential indirect-increment loop over edges 0..E-1 in order.
 * x[N][2], q[C][4], adt[C], res[C][4] row-major; e2n[E][2], e2c[E][2].
 * res is accumulated into (the caller zeroes it for a plain evaluation).
 */
void oracle_edge_loop(int64_t E, const int32_t *e2n, const int32_t *e2c,
                      const double *x, const double *q, const double *adt,
                      double gm1, double eps, double *res)
{
    for (int64_t e = 0; e < E; ++e) {
        int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        int32_t L = e2c[2 * e], R = e2c[2 * e + 1];
        double f[4];
        oracle_lf2d_flux(x + 2 * (int64_t)a, x + 2 * (int64_t)b,
                         q + 4 * (int64_t)L, q + 4 * (int64_t)R,
                         adt[L], adt[R], gm1, eps, f);
        for (int k = 0; k < 4; ++k) {
            res[4 * (int64_t)L + k] += f[k];
            res[4 * (int64_t)R + k] -= f[k];
        }
    }
}

/* Per-edge flux values f[E][4], no scatter (for per-edge comparisons). */
void oracle_edge_fluxes(int64_t E, const int32_t *e2n, const int32_t *e2c,
                        const double *x, const double *q, const double *adt,
                        double gm1, double eps, double *f_out)
{
    for (int64_t e = 0; e < E; ++e) {
        int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        int32_t L = e2c[2 * e], R = e2c[2 * e + 1];
        oracle_lf2d_flux(x + 2 * (int64_t)a, x + 2 * (int64_t)b,
                         q + 4 * (int64_t)L, q + 4 * (int64_t)R,
                         adt[L], adt[R], gm1, eps, f_out + 4 * e);
    }
}

/*
 * First-fit greedy colouring (the reading used for global, block and thread
 * colouring, Section 2.2 "Shared memory approach"): elements are visited in
 * the given order and each gets the smallest colour not already taken by an
 * earlier element that writes one of the same points.
 *
 * Element i writes points pts[off[i] .. off[i+1]).  Points are 0..npts-1.
 * Returns the number of colours, or -1 if a colour would exceed max_colours.
 * Scratch: used_head[npts] (int64, set to -1 by this function), link/col
 * arrays of length off[n] hold, per point, a singly linked list of the
 * colours already used there.
 */
int32_t oracle_first_fit(int64_t n, const int64_t *off, const int32_t *pts,
                         int64_t npts, int32_t max_colours, int32_t *colour,
                         int64_t *used_head, int64_t *link, int32_t *used_col,
                         int64_t *forbid_stamp)
{
    for (int64_t p = 0; p < npts; ++p) used_head[p] = -1;
    for (int32_t c = 0; c < max_colours + 1; ++c) forbid_stamp[c] = -1;
    int64_t nlinks = 0;
    int32_t ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            for (int64_t l = used_head[pts[k]]; l >= 0; l = link[l])
                forbid_stamp[used_col[l]] = i;
        }
        int32_t c = 0;
        while (c <= max_colours && forbid_stamp[c] == i) ++c;
        if (c >= max_colours) return -1;
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            /* a point written twice by the same element records c once */
            int dup = 0;
            for (int64_t l = used_head[pts[k]]; l >= 0; l = link[l])
                if (used_col[l] == c) { dup = 1; break; }
            if (dup) continue;
            used_col[nlinks] = c;
            link[nlinks] = used_head[pts[k]];
            used_head[pts[k]] = nlinks;
            ++nlinks;
        }
    }
    return ncol;
}

/*
 * Binary32 evaluation of the same flux (test infrastructure for the FP32
 * storage variant): inputs are binary32, every operation is one correctly
 * rounded binary32 operation in the order of oracle_lf2d_flux, gm1 is the
 * binary32 value nearest the binary64 gm1.  The loop accumulates each
 * binary32 flux, converted exactly to binary64, into a binary64 residual.
 */
static void oracle_side_flux_f32(const float *q, float nx, float ny, float gm1, float F[4])
{
    float ri = 1.0f / q[0];
    float u = q[1] * ri;
    float v = q[2] * ri;
    float p = gm1 * (q[3] - 0.5f * (q[1] * u + q[2] * v));
    float U = u * nx + v * ny;
    F[0] = q[0] * U;
    F[1] = q[1] * U + p * nx;
    F[2] = q[2] * U + p * ny;
    F[3] = (q[3] + p) * U;
}

void oracle_lf2d_flux_f32(const float *xa, const float *xb, const float *qL, const float *qR,
                          float adtL, float adtR, float gm1, float eps, float *f)
{
    float nx = xb[1] - xa[1];
    float ny = xa[0] - xb[0];
    float FL[4], FR[4];
    oracle_side_flux_f32(qL, nx, ny, gm1, FL);
    oracle_side_flux_f32(qR, nx, ny, gm1, FR);
    float mu = eps * 0.5f * (adtL + adtR);
    for (int k = 0; k < 4; ++k)
        f[k] = 0.5f * (FL[k] + FR[k]) + 0.5f * mu * (qL[k] - qR[k]);
}

void oracle_edge_loop_f32(int64_t E, const int32_t *e2n, const int32_t *e2c, const float *x,
                          const float *q, const float *adt, double gm1, double eps, double *res,
                          double *f_out)
{
    const float g = (float)gm1, ep = (float)eps;
    for (int64_t e = 0; e < E; ++e) {
        int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        int32_t L = e2c[2 * e], R = e2c[2 * e + 1];
        float f[4];
        oracle_lf2d_flux_f32(x + 2 * (int64_t)a, x + 2 * (int64_t)b, q + 4 * (int64_t)L,
                             q + 4 * (int64_t)R, adt[L], adt[R], g, ep, f);
        for (int k = 0; k < 4; ++k) {
            if (res) {
                res[4 * (int64_t)L + k] += (double)f[k];
                res[4 * (int64_t)R + k] -= (double)f[k];
            }
            if (f_out) f_out[4 * e + k] = (double)f[k];
        }
    }
}
