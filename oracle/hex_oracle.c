/*
 * CPU ORACLE -- test infrastructure, not part of the product path.
 *
 * Sequential binary64 evaluation of the 3D element loop: for every hexahedral
 * element, read the coordinates and velocities of its 8 nodes through the
 * element->node map, compute an hourglass-type nodal force and increment the
 * force of all 8 nodes (the access pattern of the LULESH stress/hourglass
 * loop, paper Section 3.1.4; the paper prints no formula, so the force is
 * our own, built on the Flanagan-Belytschko hourglass base vectors):
 *
 *   G_1 = ( 1,  1, -1, -1, -1, -1,  1,  1)
 *   G_2 = ( 1, -1, -1,  1, -1,  1,  1, -1)
 *   G_3 = ( 1, -1,  1, -1,  1, -1,  1, -1)
 *   G_4 = (-1,  1, -1,  1,  1, -1,  1, -1)
 *   h   = |x_6 - x_0|                       (main diagonal length)
 *   for each component d: m_i = sum_b G_i,b v_b,d   (b = 0..7 in order)
 *   f_a,d = (-kappa h) * (G_1,a m_1 + G_2,a m_2 + G_3,a m_3 + G_4,a m_4)
 *   force[node_a] += f_a
 *
 * Every G is +-1, so each product is a sign change; sums are taken left to
 * right in the order written.  Built -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>

static const int HG[4][8] = {{1, 1, -1, -1, -1, -1, 1, 1},
                             {1, -1, -1, 1, -1, 1, 1, -1},
                             {1, -1, 1, -1, 1, -1, 1, -1},
                             {-1, 1, -1, 1, 1, -1, 1, -1}};

static double signed_term(int s, double v) { return s > 0 ? v : -v; }

void oracle_hex_force(const double *x /* [8][3] */, const double *v /* [8][3] */, double kappa,
                      double *f /* [8][3] */)
{
    double dx = x[6 * 3 + 0] - x[0];
    double dy = x[6 * 3 + 1] - x[1];
    double dz = x[6 * 3 + 2] - x[2];
    double h = sqrt(dx * dx + dy * dy + dz * dz);
    double c = -kappa * h;
    for (int d = 0; d < 3; ++d) {
        double m[4];
        for (int i = 0; i < 4; ++i) {
            double s = signed_term(HG[i][0], v[0 * 3 + d]);
            for (int b = 1; b < 8; ++b) s = s + signed_term(HG[i][b], v[b * 3 + d]);
            m[i] = s;
        }
        for (int a = 0; a < 8; ++a) {
            double s = signed_term(HG[0][a], m[0]);
            for (int i = 1; i < 4; ++i) s = s + signed_term(HG[i][a], m[i]);
            f[a * 3 + d] = c * s;
        }
    }
}

/* Sequential element loop; force[N][3] is accumulated into.  f_out (may be
 * NULL) receives the per-element forces [E][8][3]. */
void oracle_hex_loop(int64_t E, const int32_t *e2n, const double *x, const double *v,
                     double kappa, double *force, double *f_out)
{
    for (int64_t e = 0; e < E; ++e) {
        double xe[24], ve[24], fe[24];
        for (int a = 0; a < 8; ++a) {
            int32_t n = e2n[8 * e + a];
            for (int d = 0; d < 3; ++d) {
                xe[a * 3 + d] = x[3 * (int64_t)n + d];
                ve[a * 3 + d] = v[3 * (int64_t)n + d];
            }
        }
        oracle_hex_force(xe, ve, kappa, fe);
        for (int a = 0; a < 8; ++a) {
            int32_t n = e2n[8 * e + a];
            for (int d = 0; d < 3; ++d) {
                if (force) force[3 * (int64_t)n + d] += fe[a * 3 + d];
                if (f_out) f_out[24 * e + a * 3 + d] = fe[a * 3 + d];
            }
        }
    }
}
