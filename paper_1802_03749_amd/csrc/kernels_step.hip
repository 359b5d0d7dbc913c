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

template <int LAYOUT>
__global__ __launch_bounds__(1024) void adt_kernel(const double *__restrict__ x,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ adt,
                                                   const int4 *__restrict__ c2n, int64_t N,
                                                   int64_t C, double gm1) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int4 nd = c2n[c];
    double px[4], py[4];
    load2<LAYOUT>(x, N, nd.x, px[0], py[0]);
    load2<LAYOUT>(x, N, nd.y, px[1], py[1]);
    load2<LAYOUT>(x, N, nd.z, px[2], py[2]);
    load2<LAYOUT>(x, N, nd.w, px[3], py[3]);
    double qc[4];
    load4<LAYOUT>(q, C, c, qc);
    const double ri = 1.0 / qc[0];
    const double u = qc[1] * ri;
    const double v = qc[2] * ri;
    const double p = gm1 * (qc[3] - 0.5 * (qc[1] * u + qc[2] * v));
    const double cs = sqrt((1.0 + gm1) * p * ri);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const double mx = py[k1] - py[k];
        const double my = px[k] - px[k1];
        s = s + (fabs(u * mx + v * my) + cs * sqrt(mx * mx + my * my));
    }
    adt[c] = s;
}

template <int LAYOUT, bool ATOMIC>
__global__ __launch_bounds__(1024) void bres_kernel(const double *__restrict__ x,
                                                    const double *__restrict__ q,
                                                    const double *__restrict__ adt,
                                                    double *__restrict__ res,
                                                    const int4 *__restrict__ emap, int32_t begin,
                                                    int32_t end, int64_t N, int64_t C, double gm1,
                                                    double eps, double qi0, double qi1, double qi2,
                                                    double qi3) {
    const int64_t s = begin + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= end) return;
    const int4 m = emap[s];
    const int c = m.x;
    double qc[4], xa0, xa1, xb0, xb1;
    load4<LAYOUT>(q, C, c, qc);
    load2<LAYOUT>(x, N, m.y, xa0, xa1);
    load2<LAYOUT>(x, N, m.z, xb0, xb1);
    const double a = adt[c];
    const double qi[4] = {qi0, qi1, qi2, qi3};
    double f[4];
    lf2d_flux<double>(xa0, xa1, xb0, xb1, qc, qi, a, a, gm1, eps, f);
    if constexpr (ATOMIC) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            unsafeAtomicAdd(LAYOUT == UM_AOS ? &res[4 * int64_t(c) + k] : &res[k * C + c], f[k]);
    } else {
        double r[4];
        load4<LAYOUT>(res, C, c, r);
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] += f[k];
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

template <int LAYOUT>
__global__ __launch_bounds__(1024) void update_kernel(double *__restrict__ q,
                                                      double *__restrict__ res,
                                                      const double *__restrict__ adt,
                                                      double *__restrict__ partials, int64_t C) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (c < C) {
        double qc[4], r[4];
        load4<LAYOUT>(q, C, c, qc);
        load4<LAYOUT>(res, C, c, r);
        const double a = adt[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double d = r[k] / a;
            qc[k] = qc[k] - d;
            acc = acc + d * d;
            r[k] = 0.0;
        }
        store4<LAYOUT>(q, C, c, qc);
        store4<LAYOUT>(res, C, c, r);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void reduce_kernel(const double *__restrict__ partials,
                                                      int32_t n, double *__restrict__ gbl) {
    double acc = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) gbl[0] += t;
}

int32_t grid_for(int64_t n, int32_t bs) { return int32_t((n + bs - 1) / bs); }

template <int LAYOUT>
hipError_t launch_layout(const LaunchArgs &la, int32_t kernel, int which, int32_t begin,
                         int32_t end) {
    const int32_t bs = la.block_size;
    const double *x = static_cast<const double *>(la.x);
    const double *q = static_cast<const double *>(la.q);
    const double *adt = static_cast<const double *>(la.adt);
    const int64_t n = int64_t(end) - begin;
    if (n <= 0) return hipSuccess;
    if (kernel == UM_K_CELL_ADT_2D && which == LAUNCH_DIRECT) {
        adt_kernel<LAYOUT><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, const_cast<double *>(adt), reinterpret_cast<const int4 *>(la.emap), la.N, la.C,
            la.gm1);
    } else if (kernel == UM_K_BOUNDARY_FLUX_2D && which == LAUNCH_GCOL) {
        bres_kernel<LAYOUT, false><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, adt, la.res, reinterpret_cast<const int4 *>(la.emap), begin, end, la.N, la.C,
            la.gm1, la.eps, la.qinf[0], la.qinf[1], la.qinf[2], la.qinf[3]);
    } else if (kernel == UM_K_BOUNDARY_FLUX_2D && which == LAUNCH_ATOMIC) {
        bres_kernel<LAYOUT, true><<<grid_for(n, bs), bs, 0, la.stream>>>(
            x, q, adt, la.res, reinterpret_cast<const int4 *>(la.emap), begin, end, la.N, la.C,
            la.gm1, la.eps, la.qinf[0], la.qinf[1], la.qinf[2], la.qinf[3]);
    } else if (kernel == UM_K_UPDATE_2D && which == LAUNCH_DIRECT) {
        if (grid_for(n, bs) != la.n_partials) return hipErrorInvalidValue;
        update_kernel<LAYOUT><<<la.n_partials, bs, 0, la.stream>>>(
            const_cast<double *>(q), la.res, adt, la.partials, la.C);
    } else if (kernel == UM_K_UPDATE_2D && which == LAUNCH_REDUCE) {
        reduce_kernel<<<1, 1024, 0, la.stream>>>(la.partials, la.n_partials, la.gbl);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t step_launch_one(const LaunchArgs &la, int32_t kernel, int which, int32_t begin,
                           int32_t end) {
    return la.layout == UM_AOS ? launch_layout<UM_AOS>(la, kernel, which, begin, end)
                               : launch_layout<UM_SOA>(la, kernel, which, begin, end);
}

}  // namespace um
