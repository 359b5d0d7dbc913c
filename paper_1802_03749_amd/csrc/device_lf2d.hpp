// Device helpers of the 2D finite-volume loops: the edge flux (formula in
// umesh.h, UM_K_EDGE_FLUX_LF2D) and element loads/stores of dim-2 and dim-4
// dats in AoS or SoA layout.  Included by the HIP kernel files only.
#pragma once

#include <hip/hip_runtime.h>

#include "umesh.h"

namespace um {
namespace dev {

// Flux through an edge from cell L into cell R (formula in umesh.h),
// evaluated in type Real.
#define UM_LF2D_FLUX_BODY                                                      \
    const Real half = Real(0.5), one = Real(1);                                \
    const Real nx = xb1 - xa1;                                                 \
    const Real ny = xa0 - xb0;                                                 \
    Real FL[4], FR[4];                                                         \
    {                                                                          \
        const Real ri = one / qL[0];                                           \
        const Real u = qL[1] * ri;                                             \
        const Real v = qL[2] * ri;                                             \
        const Real p = gm1 * (qL[3] - half * (qL[1] * u + qL[2] * v));         \
        const Real U = u * nx + v * ny;                                        \
        FL[0] = qL[0] * U;                                                     \
        FL[1] = qL[1] * U + p * nx;                                            \
        FL[2] = qL[2] * U + p * ny;                                            \
        FL[3] = (qL[3] + p) * U;                                               \
    }                                                                          \
    {                                                                          \
        const Real ri = one / qR[0];                                           \
        const Real u = qR[1] * ri;                                             \
        const Real v = qR[2] * ri;                                             \
        const Real p = gm1 * (qR[3] - half * (qR[1] * u + qR[2] * v));         \
        const Real U = u * nx + v * ny;                                        \
        FR[0] = qR[0] * U;                                                     \
        FR[1] = qR[1] * U + p * nx;                                            \
        FR[2] = qR[2] * U + p * ny;                                            \
        FR[3] = (qR[3] + p) * U;                                               \
    }                                                                          \
    const Real mu = eps * half * (adtL + adtR);                                \
    _Pragma("unroll") for (int k = 0; k < 4; ++k)                              \
        f[k] = half * (FL[k] + FR[k]) + half * mu * (qL[k] - qR[k]);

template <typename Real>
__device__ __forceinline__ void lf2d_flux(Real xa0, Real xa1, Real xb0, Real xb1,
                                          const Real qL[4], const Real qR[4], Real adtL,
                                          Real adtR, Real gm1, Real eps, Real f[4]) {
    UM_LF2D_FLUX_BODY
}

template <typename Real>
__device__ __forceinline__ void lf2d_flux_nocontract(Real xa0, Real xa1, Real xb0, Real xb1,
                                                     const Real qL[4], const Real qR[4],
                                                     Real adtL, Real adtR, Real gm1, Real eps,
                                                     Real f[4]) {
#pragma clang fp contract(off)
    UM_LF2D_FLUX_BODY
}

// Element g of a dim-4 / dim-2 dat in AoS ([n][dim]) or SoA ([dim][n])
// layout; AoS uses 16-byte vector loads.
template <int LAYOUT, typename Real>
__device__ __forceinline__ void load4(const Real *__restrict__ a, int64_t n, int64_t g,
                                      Real v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        if constexpr (sizeof(Real) == 8) {
            const double2 *p = reinterpret_cast<const double2 *>(a + 4 * g);
            const double2 lo = p[0], hi = p[1];
            v[0] = lo.x; v[1] = lo.y; v[2] = hi.x; v[3] = hi.y;
        } else {
            const float4 t = reinterpret_cast<const float4 *>(a)[g];
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        }
    } else {
        v[0] = a[g]; v[1] = a[n + g]; v[2] = a[2 * n + g]; v[3] = a[3 * n + g];
    }
}

template <int LAYOUT>
__device__ __forceinline__ void store4(double *__restrict__ a, int64_t n, int64_t g,
                                       const double v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        double2 *p = reinterpret_cast<double2 *>(a + 4 * g);
        p[0] = make_double2(v[0], v[1]);
        p[1] = make_double2(v[2], v[3]);
    } else {
        a[g] = v[0]; a[n + g] = v[1]; a[2 * n + g] = v[2]; a[3 * n + g] = v[3];
    }
}

template <int LAYOUT, typename Real>
__device__ __forceinline__ void load2(const Real *__restrict__ a, int64_t n, int64_t g, Real &v0,
                                      Real &v1) {
    if constexpr (LAYOUT == UM_AOS) {
        if constexpr (sizeof(Real) == 8) {
            const double2 t = reinterpret_cast<const double2 *>(a)[g];
            v0 = t.x; v1 = t.y;
        } else {
            const float2 t = reinterpret_cast<const float2 *>(a)[g];
            v0 = t.x; v1 = t.y;
        }
    } else {
        v0 = a[g]; v1 = a[n + g];
    }
}

}  // namespace dev
}  // namespace um
