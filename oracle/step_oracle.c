/*
 * CPU ORACLE -- test infrastructure, not part of the product path.
 *
 * The other loops of one explicit time step of the 2D finite-volume solver
 * whose edge loop is in flux_oracle.c (the paper's Airfoil application has
 * the loops adt_calc, res_calc, bres_calc and update, Section 3.1.1; their
 * formulas are not printed, so these are our own definitions):
 *
 * adt loop (cells, reads 4 nodes through cell->node):
 *   per counter-clockwise side k: m = (y_k+1 - y_k, x_k - x_k+1) (outward)
 *   u = q1/q0, v = q2/q0, p = gm1 (q3 - 0.5 (q1 u + q2 v)),
 *   c = sqrt((1 + gm1) p / q0)
 *   adt = sum_k ( |u m_x + v m_y| + c sqrt(m_x^2 + m_y^2) )
 * boundary flux loop (boundary edges, reads 2 nodes and 1 cell, increments
 *   the cell): the edge flux of flux_oracle.c between the cell's state (left)
 *   and a far-field state q_inf (right), both sides using the cell's adt;
 *   res[cell] += f.
 * update loop (cells): d_k = res_k / adt; q_k = q_k - d_k; res_k = 0;
 *   rms += sum_k d_k^2, accumulated over cells in order.
 *
 * Built -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>

void oracle_lf2d_flux(const double *xa, const double *xb, const double *qL, const double *qR,
                      double adtL, double adtR, double gm1, double eps, double *f);

double oracle_cell_adt(const double *xc /* [4][2] ccw */, const double *q, double gm1)
{
    double ri = 1.0 / q[0];
    double u = q[1] * ri;
    double v = q[2] * ri;
    double p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    double c = sqrt((1.0 + gm1) * p * ri);
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double *a = xc + 2 * k, *b = xc + 2 * ((k + 1) % 4);
        double mx = b[1] - a[1];
        double my = a[0] - b[0];
        s = s + (fabs(u * mx + v * my) + c * sqrt(mx * mx + my * my));
    }
    return s;
}

void oracle_adt_loop(int64_t C, const int32_t *c2n, const double *x, const double *q, double gm1,
                     double *adt)
{
    for (int64_t c = 0; c < C; ++c) {
        double xc[8];
        for (int k = 0; k < 4; ++k) {
            xc[2 * k] = x[2 * (int64_t)c2n[4 * c + k]];
            xc[2 * k + 1] = x[2 * (int64_t)c2n[4 * c + k] + 1];
        }
        adt[c] = oracle_cell_adt(xc, q + 4 * c, gm1);
    }
}

void oracle_bres_loop(int64_t B, const int32_t *b2n, const int32_t *b2c, const double *x,
                      const double *q, const double *adt, const double *qinf, double gm1,
                      double eps, double *res)
{
    for (int64_t e = 0; e < B; ++e) {
        int32_t a = b2n[2 * e], b = b2n[2 * e + 1], c = b2c[e];
        double f[4];
        oracle_lf2d_flux(x + 2 * (int64_t)a, x + 2 * (int64_t)b, q + 4 * (int64_t)c, qinf, adt[c],
                         adt[c], gm1, eps, f);
        for (int k = 0; k < 4; ++k) res[4 * (int64_t)c + k] += f[k];
    }
}

double oracle_update_loop(int64_t C, double *q, double *res, const double *adt)
{
    double rms = 0.0;
    for (int64_t c = 0; c < C; ++c)
        for (int k = 0; k < 4; ++k) {
            double d = res[4 * c + k] / adt[c];
            q[4 * c + k] = q[4 * c + k] - d;
            res[4 * c + k] = 0.0;
            rms = rms + d * d;
        }
    return rms;
}

/*
 * Binary32 storage variant of the same loops (reference of the FP32 time
 * step): x, q, adt and qinf are binary32 and the cell adt and the boundary
 * flux are evaluated in binary32; res and the update's arithmetic are
 * binary64 (d = res / adt in binary64, q rounded once to binary32), and the
 * sum of squares is binary64.
 */
void oracle_lf2d_flux_f32(const float *xa, const float *xb, const float *qL, const float *qR,
                          float adtL, float adtR, float gm1, float eps, float *f);

float oracle_cell_adt_f32(const float *xc, const float *q, float gm1)
{
    float ri = 1.0f / q[0];
    float u = q[1] * ri;
    float v = q[2] * ri;
    float p = gm1 * (q[3] - 0.5f * (q[1] * u + q[2] * v));
    float c = sqrtf((1.0f + gm1) * p * ri);
    float s = 0.0f;
    for (int k = 0; k < 4; ++k) {
        const float *a = xc + 2 * k, *b = xc + 2 * ((k + 1) % 4);
        float mx = b[1] - a[1];
        float my = a[0] - b[0];
        s = s + (fabsf(u * mx + v * my) + c * sqrtf(mx * mx + my * my));
    }
    return s;
}

void oracle_adt_loop_f32(int64_t C, const int32_t *c2n, const float *x, const float *q, double gm1,
                         float *adt)
{
    const float g = (float)gm1;
    for (int64_t c = 0; c < C; ++c) {
        float xc[8];
        for (int k = 0; k < 4; ++k) {
            xc[2 * k] = x[2 * (int64_t)c2n[4 * c + k]];
            xc[2 * k + 1] = x[2 * (int64_t)c2n[4 * c + k] + 1];
        }
        adt[c] = oracle_cell_adt_f32(xc, q + 4 * c, g);
    }
}

void oracle_bres_loop_f32(int64_t B, const int32_t *b2n, const int32_t *b2c, const float *x,
                          const float *q, const float *adt, const float *qinf, double gm1,
                          double eps, double *res)
{
    const float g = (float)gm1, ep = (float)eps;
    for (int64_t e = 0; e < B; ++e) {
        int32_t a = b2n[2 * e], b = b2n[2 * e + 1], c = b2c[e];
        float f[4];
        oracle_lf2d_flux_f32(x + 2 * (int64_t)a, x + 2 * (int64_t)b, q + 4 * (int64_t)c, qinf,
                             adt[c], adt[c], g, ep, f);
        for (int k = 0; k < 4; ++k) res[4 * (int64_t)c + k] += (double)f[k];
    }
}

double oracle_update_loop_f32(int64_t C, float *q, double *res, const float *adt)
{
    double rms = 0.0;
    for (int64_t c = 0; c < C; ++c)
        for (int k = 0; k < 4; ++k) {
            double d = res[4 * c + k] / (double)adt[c];
            q[4 * c + k] = (float)((double)q[4 * c + k] - d);
            res[4 * c + k] = 0.0;
            rms = rms + d * d;
        }
    return rms;
}
