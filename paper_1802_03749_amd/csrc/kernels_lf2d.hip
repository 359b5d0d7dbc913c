// gfx950 kernels of the 2D edge-flux indirect-increment loop.
//
//  hier_kernel   two-layer colouring (paper Section 2.2, Algorithm 1): one
//                workgroup per block, one lane per edge.  The block's staged
//                cells and nodes are gathered into LDS (structure-of-arrays
//                inside LDS), the residuals of the staged cells are preloaded
//                as the increment accumulators, every lane computes its
//                edge's flux into registers, increments are applied to LDS
//                one thread colour at a time with a workgroup barrier after
//                each colour, and the accumulators are stored back once.
//                Blocks of one block colour write disjoint cells, so a launch
//                per block colour needs no atomics.
//  gcol_kernel   global colouring baseline (Section 2.1): one launch per
//                colour, gather through the int32 maps, plain read-modify-
//                write of res.
//  atomic_kernel atomics baseline (Section 2.1): one launch, hardware FP64
//                atomic adds on res.
//  debug_kernel  per-edge fluxes with floating-point contraction disabled.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "launch.hpp"

namespace um {
namespace {

// Flux through an edge from cell L into cell R (formula in umesh.h).
#define UM_LF2D_FLUX_BODY                                                      \
    const double nx = xb1 - xa1;                                               \
    const double ny = xa0 - xb0;                                               \
    double FL[4], FR[4];                                                       \
    {                                                                          \
        const double ri = 1.0 / qL[0];                                         \
        const double u = qL[1] * ri;                                           \
        const double v = qL[2] * ri;                                           \
        const double p = gm1 * (qL[3] - 0.5 * (qL[1] * u + qL[2] * v));       \
        const double U = u * nx + v * ny;                                      \
        FL[0] = qL[0] * U;                                                     \
        FL[1] = qL[1] * U + p * nx;                                            \
        FL[2] = qL[2] * U + p * ny;                                            \
        FL[3] = (qL[3] + p) * U;                                               \
    }                                                                          \
    {                                                                          \
        const double ri = 1.0 / qR[0];                                         \
        const double u = qR[1] * ri;                                           \
        const double v = qR[2] * ri;                                           \
        const double p = gm1 * (qR[3] - 0.5 * (qR[1] * u + qR[2] * v));       \
        const double U = u * nx + v * ny;                                      \
        FR[0] = qR[0] * U;                                                     \
        FR[1] = qR[1] * U + p * nx;                                            \
        FR[2] = qR[2] * U + p * ny;                                            \
        FR[3] = (qR[3] + p) * U;                                               \
    }                                                                          \
    const double mu = eps * 0.5 * (adtL + adtR);                               \
    _Pragma("unroll") for (int k = 0; k < 4; ++k)                              \
        f[k] = 0.5 * (FL[k] + FR[k]) + 0.5 * mu * (qL[k] - qR[k]);

__device__ __forceinline__ void lf2d_flux(double xa0, double xa1, double xb0, double xb1,
                                          const double qL[4], const double qR[4], double adtL,
                                          double adtR, double gm1, double eps, double f[4]) {
    UM_LF2D_FLUX_BODY
}

__device__ __forceinline__ void lf2d_flux_nocontract(double xa0, double xa1, double xb0,
                                                     double xb1, const double qL[4],
                                                     const double qR[4], double adtL,
                                                     double adtR, double gm1, double eps,
                                                     double f[4]) {
#pragma clang fp contract(off)
    UM_LF2D_FLUX_BODY
}

// Element g of a dim-4 / dim-2 / dim-1 FP64 dat in AoS ([n][dim]) or SoA
// ([dim][n]) layout.
template <int LAYOUT>
__device__ __forceinline__ void load4(const double *__restrict__ a, int64_t n, int64_t g,
                                      double v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        const double2 *p = reinterpret_cast<const double2 *>(a + 4 * g);
        const double2 lo = p[0], hi = p[1];
        v[0] = lo.x; v[1] = lo.y; v[2] = hi.x; v[3] = hi.y;
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

template <int LAYOUT>
__device__ __forceinline__ void load2(const double *__restrict__ a, int64_t n, int64_t g,
                                      double &v0, double &v1) {
    if constexpr (LAYOUT == UM_AOS) {
        const double2 t = reinterpret_cast<const double2 *>(a)[g];
        v0 = t.x; v1 = t.y;
    } else {
        v0 = a[g]; v1 = a[n + g];
    }
}

// LDS floating-point add without return (ds_add_f64).  Inside one colour
// round no two lanes touch the same address, so the result equals a plain
// read-modify-write and stays deterministic; it is one LDS instruction
// instead of a read and a write.
__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct Dats {
    const double *__restrict__ x;
    const double *__restrict__ q;
    const double *__restrict__ adt;
    double *__restrict__ res;
    int64_t N, C;
};

template <int LAYOUT>
__device__ __forceinline__ void edge_flux_global(const Dats &d, int L, int R, int a, int b,
                                                 double gm1, double eps, double f[4]) {
    double qL[4], qR[4], xa0, xa1, xb0, xb1;
    load4<LAYOUT>(d.q, d.C, L, qL);
    load4<LAYOUT>(d.q, d.C, R, qR);
    load2<LAYOUT>(d.x, d.N, a, xa0, xa1);
    load2<LAYOUT>(d.x, d.N, b, xb0, xb1);
    const double adtL = d.adt[L], adtR = d.adt[R];
    lf2d_flux(xa0, xa1, xb0, xb1, qL, qR, adtL, adtR, gm1, eps, f);
}

// Stage the residual (as accumulator) and, when staging all, q and adt of
// staged cell t into LDS, from registers loaded by fetch_cell.
struct CellRegs {
    double r[4], q[4], a;
};

template <int LAYOUT, int STAGING>
__device__ __forceinline__ void fetch_cell(const Dats &d, int64_t g, CellRegs &c) {
    load4<LAYOUT>(d.res, d.C, g, c.r);
    if constexpr (STAGING == UM_STAGE_ALL) {
        load4<LAYOUT>(d.q, d.C, g, c.q);
        c.a = d.adt[g];
    }
}

template <int STAGING>
__device__ __forceinline__ void put_cell(double *s_inc, double *s_q, double *s_adt, int nc, int t,
                                         const CellRegs &c) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_inc[k * nc + t] = c.r[k];
    if constexpr (STAGING == UM_STAGE_ALL) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_q[k * nc + t] = c.q[k];
        s_adt[t] = c.a;
    }
}

// Point id at staged position t of a block: from the block's run
// descriptors (uniform, scalar loads) when it has any, else from its explicit
// list.  Runs are ordered by `local`, the first one starts at 0.
__device__ __forceinline__ int32_t staged_id(const Run *__restrict__ runs, int r0, int nr,
                                             const int32_t *__restrict__ list, int t) {
    if (nr == 0) return list[t];
    int32_t g = runs[r0].start + t;
    for (int r = 1; r < nr; ++r) {
        const Run R = runs[r0 + r];
        if (t >= R.local) g = R.start + (t - R.local);
    }
    return g;
}

// EPT = elements (edges) per lane: the workgroup has T lanes and handles a
// block of up to EPT*T edges; lane l computes slots l, l+T, ...
template <int LAYOUT, int STAGING, int TCMODE, int EPT>
__global__ __launch_bounds__(1024) void hier_kernel(const BlockInfo *__restrict__ binfo,
                                                    const int32_t *__restrict__ stg_c,
                                                    const int32_t *__restrict__ stg_n,
                                                    const Run *__restrict__ crun,
                                                    const Run *__restrict__ nrun,
                                                    const uint2 *__restrict__ loc, Dats d,
                                                    double gm1, double eps, int32_t base) {
    extern __shared__ double lds[];
    const int32_t pos = base + int32_t(blockIdx.x);
    const BlockInfo bi = binfo[pos], bn = binfo[pos + 1];
    const int ne = bn.slot_off - bi.slot_off;
    const int nc = bn.cell_off - bi.cell_off;
    const int nn = bn.node_off - bi.node_off;
    const int ncr = bn.crun_off - bi.crun_off, nnr = bn.nrun_off - bi.nrun_off;
    const int32_t *__restrict__ sc = stg_c + bi.cell_off;
    const int32_t *__restrict__ sn = stg_n + bi.node_off;
    auto cell_id = [&](int t) { return staged_id(crun, bi.crun_off, ncr, sc, t); };
    auto node_id = [&](int t) { return staged_id(nrun, bi.nrun_off, nnr, sn, t); };
    double *s_inc = lds;            // [4][nc] increment accumulators
    double *s_q = s_inc + 4 * nc;   // [4][nc]
    double *s_adt = s_q + 4 * nc;   // [nc]
    double *s_x = s_adt + nc;       // [2][nn]
    const int tid = int(threadIdx.x), T = int(blockDim.x);

    // local index words of this lane's slots: issued first, used after the
    // barrier
    uint2 w[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int s = tid + j * T;
        w[j] = s < ne ? loc[bi.slot_off + s] : make_uint2(0, 0);
    }

    // gather: two staged cells and two staged nodes per lane per pass, all
    // loads of a pass issued before its LDS stores
    for (int t0 = tid; t0 < nc; t0 += 2 * T) {
        const int t1 = t0 + T;
        const bool has1 = t1 < nc;
        const int64_t g0 = cell_id(t0);
        const int64_t g1 = has1 ? cell_id(t1) : g0;
        CellRegs c0, c1;
        fetch_cell<LAYOUT, STAGING>(d, g0, c0);
        fetch_cell<LAYOUT, STAGING>(d, g1, c1);
        put_cell<STAGING>(s_inc, s_q, s_adt, nc, t0, c0);
        if (has1) put_cell<STAGING>(s_inc, s_q, s_adt, nc, t1, c1);
    }
    if constexpr (STAGING == UM_STAGE_ALL) {
        for (int t0 = tid; t0 < nn; t0 += 2 * T) {
            const int t1 = t0 + T;
            const bool has1 = t1 < nn;
            const int64_t g0 = node_id(t0);
            const int64_t g1 = has1 ? node_id(t1) : g0;
            double a0, a1, b0, b1;
            load2<LAYOUT>(d.x, d.N, g0, a0, a1);
            load2<LAYOUT>(d.x, d.N, g1, b0, b1);
            s_x[t0] = a0;
            s_x[nn + t0] = a1;
            if (has1) {
                s_x[t1] = b0;
                s_x[nn + t1] = b1;
            }
        }
    }
    __syncthreads();

    // fluxes of this lane's edges into registers
    int lL[EPT], lR[EPT], col[EPT];
    double f[EPT][4];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        lL[j] = int(w[j].x & 0x7FFu);
        col[j] = (tid + j * T) < ne ? int((w[j].x >> 11) & 31u) : -1;
        lR[j] = int((w[j].x >> 16) & 0x7FFu);
        const int nA = int(w[j].y & 0xFFFFu), nB = int(w[j].y >> 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) f[j][k] = 0.0;
        if (col[j] >= 0) {
            if constexpr (STAGING == UM_STAGE_ALL) {
                double qL[4], qR[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    qL[k] = s_q[k * nc + lL[j]];
                    qR[k] = s_q[k * nc + lR[j]];
                }
                lf2d_flux(s_x[nA], s_x[nn + nA], s_x[nB], s_x[nn + nB], qL, qR, s_adt[lL[j]],
                          s_adt[lR[j]], gm1, eps, f[j]);
            } else {
                edge_flux_global<LAYOUT>(d, cell_id(lL[j]), cell_id(lR[j]), node_id(nA),
                                         node_id(nB), gm1, eps, f[j]);
            }
        }
    }

    if constexpr (TCMODE == UM_TC_BARRIER) {
        // layer 2: one thread colour at a time; same-colour edges never share
        // a cell, so their LDS read-modify-writes do not race.  Slots are
        // sorted by colour, so most wavefronts hold a single colour.
        const int ncol = bi.ncol;
        for (int c = 0; c < ncol; ++c) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (col[j] == c) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        lds_add(&s_inc[k * nc + lL[j]], f[j][k]);
                        lds_add(&s_inc[k * nc + lR[j]], -f[j][k]);
                    }
                }
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (col[j] >= 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    lds_add(&s_inc[k * nc + lL[j]], f[j][k]);
                    lds_add(&s_inc[k * nc + lR[j]], -f[j][k]);
                }
            }
        }
        __syncthreads();
    }

    // write back once per staged cell; no other block of this colour
    // touches these cells
    for (int t = tid; t < nc; t += T) {
        double r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = s_inc[k * nc + t];
        store4<LAYOUT>(d.res, d.C, cell_id(t), r);
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void gcol_kernel(const int4 *__restrict__ emap, int32_t begin,
                                                   int32_t end, Dats d, double gm1, double eps) {
    const int32_t s = begin + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= end) return;
    const int4 m = emap[s];  // L, R, a, b
    double f[4];
    edge_flux_global<LAYOUT>(d, m.x, m.y, m.z, m.w, gm1, eps, f);
    double rL[4], rR[4];
    load4<LAYOUT>(d.res, d.C, m.x, rL);
    load4<LAYOUT>(d.res, d.C, m.y, rR);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        rL[k] += f[k];
        rR[k] -= f[k];
    }
    store4<LAYOUT>(d.res, d.C, m.x, rL);
    store4<LAYOUT>(d.res, d.C, m.y, rR);
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void atomic_kernel(const int4 *__restrict__ emap, int32_t n,
                                                     Dats d, double gm1, double eps) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int4 m = emap[s];
    double f[4];
    edge_flux_global<LAYOUT>(d, m.x, m.y, m.z, m.w, gm1, eps, f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t iL = LAYOUT == UM_AOS ? 4 * int64_t(m.x) + k : k * d.C + m.x;
        const int64_t iR = LAYOUT == UM_AOS ? 4 * int64_t(m.y) + k : k * d.C + m.y;
        unsafeAtomicAdd(&d.res[iL], f[k]);
        unsafeAtomicAdd(&d.res[iR], -f[k]);
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void debug_kernel(const int4 *__restrict__ emap, int32_t n,
                                                    Dats d, double gm1, double eps,
                                                    double *__restrict__ out) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int4 m = emap[s];
    double qL[4], qR[4], xa0, xa1, xb0, xb1, f[4];
    load4<LAYOUT>(d.q, d.C, m.x, qL);
    load4<LAYOUT>(d.q, d.C, m.y, qR);
    load2<LAYOUT>(d.x, d.N, m.z, xa0, xa1);
    load2<LAYOUT>(d.x, d.N, m.w, xb0, xb1);
    lf2d_flux_nocontract(xa0, xa1, xb0, xb1, qL, qR, d.adt[m.x], d.adt[m.y], gm1, eps, f);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * int64_t(s) + k] = f[k];
}

template <int LAYOUT, int ST, int TC, int EPT>
void set_attr_one() {
    hipFuncSetAttribute(reinterpret_cast<const void *>(hier_kernel<LAYOUT, ST, TC, EPT>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int LAYOUT, int ST, int TC>
hipError_t launch_hier_ept(const LaunchArgs &la, int32_t nblocks, int32_t base, int64_t lds,
                           Dats d) {
    static bool attrs = false;
    if (!attrs) {
        set_attr_one<LAYOUT, ST, TC, 1>();
        set_attr_one<LAYOUT, ST, TC, 2>();
        set_attr_one<LAYOUT, ST, TC, 4>();
        attrs = true;
    }
    dim3 grid(nblocks), block(la.block_size);
    const uint2 *loc = reinterpret_cast<const uint2 *>(la.loc);
    switch (la.ept) {
    case 1:
        hipLaunchKernelGGL((hier_kernel<LAYOUT, ST, TC, 1>), grid, block, size_t(lds), la.stream,
                           la.binfo, la.stg_c, la.stg_n, la.crun, la.nrun, loc, d, la.gm1,
                           la.eps, base);
        break;
    case 2:
        hipLaunchKernelGGL((hier_kernel<LAYOUT, ST, TC, 2>), grid, block, size_t(lds), la.stream,
                           la.binfo, la.stg_c, la.stg_n, la.crun, la.nrun, loc, d, la.gm1,
                           la.eps, base);
        break;
    case 4:
        hipLaunchKernelGGL((hier_kernel<LAYOUT, ST, TC, 4>), grid, block, size_t(lds), la.stream,
                           la.binfo, la.stg_c, la.stg_n, la.crun, la.nrun, loc, d, la.gm1,
                           la.eps, base);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int LAYOUT>
hipError_t launch_hier(const LaunchArgs &la, int32_t nblocks, int32_t base, int64_t lds, Dats d) {
    if (la.staging == UM_STAGE_ALL && la.tcmode == UM_TC_BARRIER)
        return launch_hier_ept<LAYOUT, UM_STAGE_ALL, UM_TC_BARRIER>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_ALL && la.tcmode == UM_TC_LDS_ATOMIC)
        return launch_hier_ept<LAYOUT, UM_STAGE_ALL, UM_TC_LDS_ATOMIC>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_INC_ONLY && la.tcmode == UM_TC_BARRIER)
        return launch_hier_ept<LAYOUT, UM_STAGE_INC_ONLY, UM_TC_BARRIER>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_INC_ONLY && la.tcmode == UM_TC_LDS_ATOMIC)
        return launch_hier_ept<LAYOUT, UM_STAGE_INC_ONLY, UM_TC_LDS_ATOMIC>(la, nblocks, base, lds, d);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t lf2d_launch_one(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                           int64_t lds) {
    Dats d{la.x, la.q, la.adt, la.res, la.N, la.C};
    const int layout = la.layout;
    if (which == LAUNCH_HIER)
        return layout == UM_AOS ? launch_hier<UM_AOS>(la, end - begin, begin, lds, d)
                                : launch_hier<UM_SOA>(la, end - begin, begin, lds, d);
    const int32_t n = end - begin;
    if (n <= 0) return hipSuccess;
    const int tb = la.block_size;
    dim3 grid((n + tb - 1) / tb), block(tb);
    const int4 *em = reinterpret_cast<const int4 *>(la.emap);
    if (which == LAUNCH_GCOL) {
        if (layout == UM_AOS)
            hipLaunchKernelGGL(gcol_kernel<UM_AOS>, grid, block, 0, la.stream, em, begin, end, d,
                               la.gm1, la.eps);
        else
            hipLaunchKernelGGL(gcol_kernel<UM_SOA>, grid, block, 0, la.stream, em, begin, end, d,
                               la.gm1, la.eps);
    } else if (which == LAUNCH_ATOMIC) {
        if (layout == UM_AOS)
            hipLaunchKernelGGL(atomic_kernel<UM_AOS>, grid, block, 0, la.stream, em, n, d, la.gm1,
                               la.eps);
        else
            hipLaunchKernelGGL(atomic_kernel<UM_SOA>, grid, block, 0, la.stream, em, n, d, la.gm1,
                               la.eps);
    } else if (which == LAUNCH_DEBUG) {
        if (layout == UM_AOS)
            hipLaunchKernelGGL(debug_kernel<UM_AOS>, grid, block, 0, la.stream, em, n, d, la.gm1,
                               la.eps, la.out);
        else
            hipLaunchKernelGGL(debug_kernel<UM_SOA>, grid, block, 0, la.stream, em, n, d, la.gm1,
                               la.eps, la.out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace um
