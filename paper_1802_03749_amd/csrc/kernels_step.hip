// gfx950 kernels of the other loops of one explicit time step of the 2D
// finite-volume solver (formulas and argument patterns in umesh.h):
//
//  adt_kernel     cell loop; gathers the 4 nodes of a cell through the
//                 cell->node map (one 16-byte load of the map row) and
//                 writes the cell's time-step scalar.  Read-only indirection,
//                 so no colouring.
//  bres_kernel    boundary-edge loop; the edge flux against the far-field
//                 state, incremented into the edge's cell.  Coloured (one
//                 launch per colour, plain read-modify-write) or with
//                 hardware FP64 atomics.
//  update_kernel  cell loop; q -= res/adt, res = 0, and a per-workgroup sum
//                 of the squared changes in a fixed reduction tree.
//  update_adt_kernel  the update, then the cell's time-step scalar from the
//                 updated state (adt_kernel's evaluation, so the same bits).
//  reduce_kernel  one workgroup adds the per-workgroup sums, in a fixed
//                 order, to the global target.
#include <hip/hip_runtime.h>

#include "device_lf2d.hpp"
#include "internal.hpp"
#include "launch.hpp"

namespace um {
namespace {

using dev::lf2d_flux;
using dev::load2;
using dev::load4;
using dev::store4;

// Store of a dim-4 element in type Real (AoS: 16-byte vector stores).
template <int LAYOUT, typename Real>
__device__ __forceinline__ void store4r(Real *__restrict__ a, int64_t n, int64_t g,
                                        const Real v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        if constexpr (sizeof(Real) == 8) {
            store4<LAYOUT>(reinterpret_cast<double *>(a), n, g, reinterpret_cast<const double *>(v));
        } else {
            reinterpret_cast<float4 *>(a)[g] = make_float4(v[0], v[1], v[2], v[3]);
        }
    } else {
        a[g] = v[0]; a[n + g] = v[1]; a[2 * n + g] = v[2]; a[3 * n + g] = v[3];
    }
}

// Time-step scalar of the cell with nodes nd and state qc, in the storage
// type Real (the one evaluation both adt kernels use).
template <int LAYOUT, typename Real>
__device__ __forceinline__ Real cell_adt(const Real *__restrict__ x, int64_t N, int4 nd,
                                         const Real qc[4], double gm1d) {
    const Real gm1 = Real(gm1d), half = Real(0.5), one = Real(1);
    Real px[4], py[4];
    load2<LAYOUT>(x, N, nd.x, px[0], py[0]);
    load2<LAYOUT>(x, N, nd.y, px[1], py[1]);
    load2<LAYOUT>(x, N, nd.z, px[2], py[2]);
    load2<LAYOUT>(x, N, nd.w, px[3], py[3]);
    const Real ri = one / qc[0];
    const Real u = qc[1] * ri;
    const Real v = qc[2] * ri;
    const Real p = gm1 * (qc[3] - half * (qc[1] * u + qc[2] * v));
    const Real cs = sqrt((one + gm1) * p * ri);
    Real s = Real(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const Real mx = py[k1] - py[k];
        const Real my = px[k] - px[k1];
        s = s + (fabs(u * mx + v * my) + cs * sqrt(mx * mx + my * my));
    }
    return s;
}

// Cell time-step scalar, evaluated in the storage type Real.
template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void adt_kernel(const Real *__restrict__ x,
                                                   const Real *__restrict__ q,
                                                   Real *__restrict__ adt,
                                                   const int4 *__restrict__ c2n, int64_t N,
                                                   int64_t C, double gm1d) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= C) return;
    Real qc[4];
    load4<LAYOUT>(q, C, c, qc);
    adt[c] = cell_adt<LAYOUT, Real>(x, N, c2n[c], qc, gm1d);
}

// Far-field boundary flux, evaluated in Real; increments in double.
template <int LAYOUT, bool ATOMIC, typename Real>
__global__ __launch_bounds__(1024) void bres_kernel(const Real *__restrict__ x,
                                                    const Real *__restrict__ q,
                                                    const Real *__restrict__ adt,
                                                    double *__restrict__ res,
                                                    const int4 *__restrict__ emap, int32_t begin,
                                                    int32_t end, int64_t N, int64_t C, double gm1,
                                                    double eps, double qi0, double qi1, double qi2,
                                                    double qi3) {
    const int64_t s = begin + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= end) return;
    const int4 m = emap[s];
    const int c = m.x;
    Real qc[4], xa0, xa1, xb0, xb1;
    load4<LAYOUT>(q, C, c, qc);
    load2<LAYOUT>(x, N, m.y, xa0, xa1);
    load2<LAYOUT>(x, N, m.z, xb0, xb1);
    const Real a = adt[c];
    const Real qi[4] = {Real(qi0), Real(qi1), Real(qi2), Real(qi3)};
    Real f[4];
    lf2d_flux<Real>(xa0, xa1, xb0, xb1, qc, qi, a, a, Real(gm1), Real(eps), f);
    if constexpr (ATOMIC) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            unsafeAtomicAdd(LAYOUT == UM_AOS ? &res[4 * int64_t(c) + k] : &res[k * C + c],
                            double(f[k]));
    } else {
        double r[4];
        load4<LAYOUT>(res, C, c, r);
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] += double(f[k]);
        store4<LAYOUT>(res, C, c, r);
    }
}

// Sum over the 64 lanes of a wave in a fixed butterfly; every lane ends
// with the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order sum over the workgroup (waves in order); valid in lane 0 of
// wave 0.  blockDim.x is a multiple of 64, at most 1024.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double wsum[16];
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wsum[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < int(blockDim.x >> 6); ++w) t += wsum[w];
    return t;
}

// Update: d = res / adt in double, q rounded once to its storage type.
template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void update_kernel(Real *__restrict__ q,
                                                      double *__restrict__ res,
                                                      const Real *__restrict__ adt,
                                                      double *__restrict__ partials, int64_t C) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (c < C) {
        Real qc[4];
        double r[4];
        load4<LAYOUT>(q, C, c, qc);
        load4<LAYOUT>(res, C, c, r);
        const double a = double(adt[c]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double d = r[k] / a;
            qc[k] = Real(double(qc[k]) - d);
            acc = acc + d * d;
            r[k] = 0.0;
        }
        store4r<LAYOUT>(q, C, c, qc);
        store4<LAYOUT>(res, C, c, r);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Update, then the next step's time-step scalar from the updated (rounded)
// state: per cell the values update_kernel and adt_kernel give in turn.
template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void update_adt_kernel(Real *__restrict__ q,
                                                          double *__restrict__ res,
                                                          Real *__restrict__ adt,
                                                          const Real *__restrict__ x,
                                                          const int4 *__restrict__ c2n,
                                                          double *__restrict__ partials,
                                                          int64_t N, int64_t C, double gm1d) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (c < C) {
        const int4 nd = c2n[c];
        Real qc[4];
        double r[4];
        load4<LAYOUT>(q, C, c, qc);
        load4<LAYOUT>(res, C, c, r);
        const double a = double(adt[c]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double d = r[k] / a;
            qc[k] = Real(double(qc[k]) - d);
            acc = acc + d * d;
            r[k] = 0.0;
        }
        store4r<LAYOUT>(q, C, c, qc);
        store4<LAYOUT>(res, C, c, r);
        adt[c] = cell_adt<LAYOUT, Real>(x, N, nd, qc, gm1d);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void reduce_kernel(const double *__restrict__ partials,
                                                      int32_t n, double *__restrict__ gbl) {
    // lane t adds partials t, t + T, t + 2T, ... in that order; the loads of
    // eight terms are issued before their additions (a zero past the end
    // leaves the non-negative sum unchanged)
    constexpr int U = 8;
    const int32_t T = int32_t(blockDim.x);
    double acc = 0.0;
    for (int32_t i0 = threadIdx.x; i0 < n; i0 += U * T) {
        double v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t i = i0 + j * T;
            v[j] = i < n ? partials[i] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) acc += v[j];
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) gbl[0] += t;
}

int32_t grid_for(int64_t n, int32_t bs) { return int32_t((n + bs - 1) / bs); }

template <int LAYOUT, typename Real>
hipError_t launch_typed(const LaunchArgs &la, int32_t kernel, int which, int32_t begin,
                        int32_t end) {
    const int32_t bs = la.block_size;
    const Real *x = static_cast<const Real *>(la.x);
    const Real *q = static_cast<const Real *>(la.q);
    const Real *adt = static_cast<const Real *>(la.adt);
    const int64_t n = int64_t(end) - begin;
    if (n <= 0) return hipSuccess;
    clear_stale_error();
    if (kernel == UM_K_CELL_ADT_2D && which == LAUNCH_DIRECT) {
        adt_kernel<LAYOUT, Real><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, const_cast<Real *>(adt), reinterpret_cast<const int4 *>(la.emap), la.N, la.C,
            la.gm1);
    } else if (kernel == UM_K_BOUNDARY_FLUX_2D && which == LAUNCH_GCOL) {
        bres_kernel<LAYOUT, false, Real><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, adt, la.res, reinterpret_cast<const int4 *>(la.emap), begin, end, la.N, la.C,
            la.gm1, la.eps, la.qinf[0], la.qinf[1], la.qinf[2], la.qinf[3]);
    } else if (kernel == UM_K_BOUNDARY_FLUX_2D && which == LAUNCH_ATOMIC) {
        bres_kernel<LAYOUT, true, Real><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, adt, la.res, reinterpret_cast<const int4 *>(la.emap), begin, end, la.N, la.C,
            la.gm1, la.eps, la.qinf[0], la.qinf[1], la.qinf[2], la.qinf[3]);
    } else if (kernel == UM_K_UPDATE_2D && which == LAUNCH_DIRECT) {
        if (grid_for(n, bs) != la.n_partials) return hipErrorInvalidValue;
        update_kernel<LAYOUT, Real><<<la.n_partials, bs, 0, la.stream>>>(
            const_cast<Real *>(q), la.res, adt, la.partials, la.C);
    } else if (kernel == UM_K_UPDATE_ADT_2D && which == LAUNCH_DIRECT) {
        if (grid_for(n, bs) != la.n_partials) return hipErrorInvalidValue;
        update_adt_kernel<LAYOUT, Real><<<la.n_partials, bs, 0, la.stream>>>(
            const_cast<Real *>(q), la.res, const_cast<Real *>(adt), x,
            reinterpret_cast<const int4 *>(la.emap), la.partials, la.N, la.C, la.gm1);
    } else if ((kernel == UM_K_UPDATE_2D || kernel == UM_K_UPDATE_ADT_2D) &&
               which == LAUNCH_REDUCE) {
        reduce_kernel<<<1, 1024, 0, la.stream>>>(la.partials, la.n_partials, la.gbl);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t step_launch_one(const LaunchArgs &la, int32_t kernel, int which, int32_t begin,
                           int32_t end) {
    if (la.dtype == UM_F32)
        return la.layout == UM_AOS ? launch_typed<UM_AOS, float>(la, kernel, which, begin, end)
                                   : launch_typed<UM_SOA, float>(la, kernel, which, begin, end);
    return la.layout == UM_AOS ? launch_typed<UM_AOS, double>(la, kernel, which, begin, end)
                               : launch_typed<UM_SOA, double>(la, kernel, which, begin, end);
}

}  // namespace um
