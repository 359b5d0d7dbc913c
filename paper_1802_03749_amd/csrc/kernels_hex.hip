// gfx950 kernels of the 3D hexahedral element loop (hourglass-type force on
// the 8 nodes of each element; formula in umesh.h, UM_K_HEX_HOURGLASS_3D).
//
//  hex_hier_kernel   two-layer colouring (paper Section 2.2, Algorithm 1):
//                    one workgroup per block of elements; the staged nodes'
//                    x, v and (as FP64 accumulators) force are gathered into
//                    LDS, every lane computes its element's 24 force values
//                    in registers, the thread colours are applied one at a
//                    time with ds_add_f64 and a barrier after each, and the
//                    accumulators are stored back once.
//  hex_gcol_kernel   global colouring: one launch per colour, plain
//                    read-modify-write of force.
//  hex_flow_kernel   the dataflow schedule: one launch, each block waits for
//                    its earlier-coloured neighbours before its write-back.
//  hex_atomic_kernel one launch, hardware FP64 atomic adds.
//  hex_debug_kernel  per-element forces with contraction disabled.
#include <hip/hip_runtime.h>

#include "device_staged.hpp"
#include "internal.hpp"
#include "launch.hpp"

namespace um {
namespace {

// v times the sign of hourglass base vector i at node a.
__device__ __forceinline__ double hg_term(int i, int a, double v) {
    // G_1 = ( 1,  1, -1, -1, -1, -1,  1,  1)
    // G_2 = ( 1, -1, -1,  1, -1,  1,  1, -1)
    // G_3 = ( 1, -1,  1, -1,  1, -1,  1, -1)
    // G_4 = (-1,  1, -1,  1,  1, -1,  1, -1)
    constexpr int G[4][8] = {{1, 1, -1, -1, -1, -1, 1, 1},
                             {1, -1, -1, 1, -1, 1, 1, -1},
                             {1, -1, 1, -1, 1, -1, 1, -1},
                             {-1, 1, -1, 1, 1, -1, 1, -1}};
    return G[i][a] > 0 ? v : -v;
}

// Forces f[a][d] of one element from its nodes' coordinates and
// velocities; sums left to right as written (same order as the definition).
#define UM_HEX_FORCE_BODY                                                     \
    const double dx = x[6][0] - x[0][0];                                      \
    const double dy = x[6][1] - x[0][1];                                      \
    const double dz = x[6][2] - x[0][2];                                      \
    const double h = sqrt(dx * dx + dy * dy + dz * dz);                       \
    const double c = -kappa * h;                                              \
    _Pragma("unroll") for (int d = 0; d < 3; ++d) {                           \
        double m[4];                                                          \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                       \
            double s = hg_term(i, 0, v[0][d]);                                \
            _Pragma("unroll") for (int b = 1; b < 8; ++b) s = s + hg_term(i, b, v[b][d]); \
            m[i] = s;                                                         \
        }                                                                     \
        _Pragma("unroll") for (int a = 0; a < 8; ++a) {                       \
            double s = hg_term(0, a, m[0]);                                   \
            _Pragma("unroll") for (int i = 1; i < 4; ++i) s = s + hg_term(i, a, m[i]); \
            f[a][d] = c * s;                                                  \
        }                                                                     \
    }

__device__ __forceinline__ void hex_force(const double x[8][3], const double v[8][3],
                                          double kappa, double f[8][3]) {
    UM_HEX_FORCE_BODY
}

__device__ __forceinline__ void hex_force_nocontract(const double x[8][3], const double v[8][3],
                                                     double kappa, double f[8][3]) {
#pragma clang fp contract(off)
    UM_HEX_FORCE_BODY
}

template <int LAYOUT>
__device__ __forceinline__ void load3(const double *__restrict__ a, int64_t n, int64_t g,
                                      double v[3]) {
    if constexpr (LAYOUT == UM_AOS) {
        v[0] = a[3 * g]; v[1] = a[3 * g + 1]; v[2] = a[3 * g + 2];
    } else {
        v[0] = a[g]; v[1] = a[n + g]; v[2] = a[2 * n + g];
    }
}

template <int LAYOUT>
__device__ __forceinline__ int64_t idx3(int64_t n, int64_t g, int d) {
    return LAYOUT == UM_AOS ? 3 * g + d : d * n + g;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct HexDats {
    const double *__restrict__ x;
    const double *__restrict__ v;
    double *__restrict__ force;
    int64_t N;
};

template <int LAYOUT, int TCMODE>
__global__ __launch_bounds__(1024) void hex_hier_kernel(const BlockInfo *__restrict__ binfo,
                                                        const int32_t *__restrict__ stg,
                                                        const Run *__restrict__ runs,
                                                        const uint4 *__restrict__ loc, HexDats d,
                                                        double kappa, int32_t base) {
    extern __shared__ double lds[];
    const int32_t pos = base + int32_t(blockIdx.x);
    const BlockInfo bi = binfo[pos], bn = binfo[pos + 1];
    const int ne = bn.slot_off - bi.slot_off;
    const int nn = bn.cell_off - bi.cell_off;
    const int nr = bn.crun_off - bi.crun_off;
    const int32_t *__restrict__ sl = stg + bi.cell_off;
    dev::StagedIds staged_id;
    staged_id.init(runs, bi.crun_off, nr, sl);
    double *s_acc = lds;           // [3][nn] force accumulators
    double *s_x = s_acc + 3 * nn;  // [3][nn]
    double *s_v = s_x + 3 * nn;    // [3][nn]
    int32_t *s_id = reinterpret_cast<int32_t *>(s_v + 3 * nn);  // [nn] staged node ids
    const int tid = int(threadIdx.x), T = int(blockDim.x);

    const uint4 w = tid < ne ? loc[bi.slot_off + tid] : make_uint4(0, 0, 0, 0);
    // gather: two staged nodes per lane per pass (a block of S elements
    // stages up to about 2 S nodes); both ids first, then all loads of the
    // pass, then its LDS stores (an id loaded after a data load would wait
    // for it).  The ids stay in LDS for the write-back.
    for (int t0 = tid; t0 < nn; t0 += 2 * T) {
        const int t1 = t0 + T;
        const bool has1 = t1 < nn;
        const int32_t g0 = staged_id(t0);
        const int32_t g1 = has1 ? staged_id(t1) : 0;
        double xv[2][3], vv[2][3], fv[2][3];
        load3<LAYOUT>(d.x, d.N, g0, xv[0]);
        load3<LAYOUT>(d.v, d.N, g0, vv[0]);
        load3<LAYOUT>(d.force, d.N, g0, fv[0]);
        if (has1) {
            load3<LAYOUT>(d.x, d.N, g1, xv[1]);
            load3<LAYOUT>(d.v, d.N, g1, vv[1]);
            load3<LAYOUT>(d.force, d.N, g1, fv[1]);
        }
        s_id[t0] = g0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_x[k * nn + t0] = xv[0][k];
            s_v[k * nn + t0] = vv[0][k];
            s_acc[k * nn + t0] = fv[0][k];
        }
        if (has1) {
            s_id[t1] = g1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s_x[k * nn + t1] = xv[1][k];
                s_v[k * nn + t1] = vv[1][k];
                s_acc[k * nn + t1] = fv[1][k];
            }
        }
    }
    __syncthreads();

    int l[8];
    l[0] = int(w.x & 0x7FFu); l[1] = int(w.x >> 16);
    l[2] = int(w.y & 0xFFFFu); l[3] = int(w.y >> 16);
    l[4] = int(w.z & 0xFFFFu); l[5] = int(w.z >> 16);
    l[6] = int(w.w & 0xFFFFu); l[7] = int(w.w >> 16);
    const int col = tid < ne ? int((w.x >> 11) & 31u) : -1;
    double f[8][3] = {};
    if (col >= 0) {
        double xe[8][3], ve[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xe[a][k] = s_x[k * nn + l[a]];
                ve[a][k] = s_v[k * nn + l[a]];
            }
        hex_force(xe, ve, kappa, f);
    }
    if constexpr (TCMODE == UM_TC_BARRIER) {
        const int ncol = bi.ncol;
        for (int c = 0; c < ncol; ++c) {
            if (col == c) {
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) lds_add(&s_acc[k * nn + l[a]], f[a][k]);
            }
            __syncthreads();
        }
    } else {
        // LDS atomics without thread colours: one round, order not fixed
        if (col >= 0) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) lds_add(&s_acc[k * nn + l[a]], f[a][k]);
        }
        __syncthreads();
    }
    for (int t = tid; t < nn; t += T) {
        const int64_t g = s_id[t];
#pragma unroll
        for (int k = 0; k < 3; ++k) d.force[idx3<LAYOUT>(d.N, g, k)] = s_acc[k * nn + t];
    }
}

// DATAFLOW schedule of the hex loop (the protocol of hier_flow_kernel in
// kernels_lf2d.hip: one launch over all blocks in colour order; a block
// gathers x and v, computes its forces and sums them per staged node in LDS
// (thread-colour rounds or LDS atomics into zeroed accumulators), waits
// until the completion flags of its earlier-coloured neighbours hold this
// execution's epoch (its own flag + 1), then adds its sums to the force
// values of its staged nodes with device-scope (sc1) loads and stores and
// publishes its flag).  With 8 block colours the sweep is a chain of 8
// blocks deep, so only the global read-add-write follows the wait.  Force
// accesses go through a buffer resource over force (24 N bytes); with AoS,
// consecutive lanes handle consecutive doubles, so one instruction covers
// whole lines of a run of consecutive nodes.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int HEX_CPOL_SC1 = 16;

template <int LAYOUT, int TCMODE>
__global__ __launch_bounds__(1024) void hex_flow_kernel(
    const BlockInfo *__restrict__ binfo, const int32_t *__restrict__ stg,
    const Run *__restrict__ runs, const uint4 *__restrict__ loc, HexDats d, double kappa,
    const int32_t *__restrict__ pred_off, const int32_t *__restrict__ preds, int32_t *flags,
    int32_t *ctl, uint64_t wait_ticks) {
    extern __shared__ double lds[];
    const int32_t pos = int32_t(blockIdx.x);
    const int32_t epoch =
        __hip_atomic_load(flags + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    const BlockInfo bi = binfo[pos], bn = binfo[pos + 1];
    const int ne = bn.slot_off - bi.slot_off;
    const int nn = bn.cell_off - bi.cell_off;
    const int nr = bn.crun_off - bi.crun_off;
    const int32_t *__restrict__ sl = stg + bi.cell_off;
    dev::StagedIds staged_id;
    staged_id.init(runs, bi.crun_off, nr, sl);
    // force accumulators [3][nn16]: inside each aligned group of 16 nodes the
    // index is swizzled (xor with the group number), so that the nodes one
    // colour round updates (a regular sublattice of a brick) spread over the
    // LDS banks instead of meeting in a few of them
    const int nn16 = (nn + 15) & ~15;
    auto ai = [nn16](int k, int l) { return k * nn16 + (l ^ ((l >> 4) & 15)); };
    double *s_acc = lds;
    double *s_x = s_acc + 3 * nn16;  // [3][nn]
    double *s_v = s_x + 3 * nn;    // [3][nn]
    int32_t *s_id = reinterpret_cast<int32_t *>(s_v + 3 * nn);  // [nn] staged node ids
    const int tid = int(threadIdx.x), T = int(blockDim.x);
    const int p0 = pred_off[pos], np = pred_off[pos + 1] - p0;

    const uint4 w = tid < ne ? loc[bi.slot_off + tid] : make_uint4(0, 0, 0, 0);
    for (int u = tid; u < 3 * nn16; u += T) s_acc[u] = 0.0;
    // both ids of a pass first, then its loads (see hex_hier_kernel); the
    // ids stay in LDS for the force accesses after the wait
    for (int t0 = tid; t0 < nn; t0 += 2 * T) {
        const int t1 = t0 + T;
        const bool has1 = t1 < nn;
        const int32_t g0 = staged_id(t0);
        const int32_t g1 = has1 ? staged_id(t1) : 0;
        double xv[2][3], vv[2][3];
        load3<LAYOUT>(d.x, d.N, g0, xv[0]);
        load3<LAYOUT>(d.v, d.N, g0, vv[0]);
        if (has1) {
            load3<LAYOUT>(d.x, d.N, g1, xv[1]);
            load3<LAYOUT>(d.v, d.N, g1, vv[1]);
        }
        s_id[t0] = g0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_x[k * nn + t0] = xv[0][k];
            s_v[k * nn + t0] = vv[0][k];
        }
        if (has1) {
            s_id[t1] = g1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s_x[k * nn + t1] = xv[1][k];
                s_v[k * nn + t1] = vv[1][k];
            }
        }
    }
    __syncthreads();

    int l[8];
    l[0] = int(w.x & 0x7FFu); l[1] = int(w.x >> 16);
    l[2] = int(w.y & 0xFFFFu); l[3] = int(w.y >> 16);
    l[4] = int(w.z & 0xFFFFu); l[5] = int(w.z >> 16);
    l[6] = int(w.w & 0xFFFFu); l[7] = int(w.w >> 16);
    const int col = tid < ne ? int((w.x >> 11) & 31u) : -1;
    double f[8][3] = {};
    if (col >= 0) {
        double xe[8][3], ve[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xe[a][k] = s_x[k * nn + l[a]];
                ve[a][k] = s_v[k * nn + l[a]];
            }
        hex_force(xe, ve, kappa, f);
    }

    // the block's sums per staged node, before the wait
    if constexpr (TCMODE == UM_TC_BARRIER) {
        const int ncol = bi.ncol;
        for (int c = 0; c < ncol; ++c) {
            if (col == c) {
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) lds_add(&s_acc[ai(k, l[a])], f[a][k]);
            }
            __syncthreads();
        }
    } else {
        if (col >= 0) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) lds_add(&s_acc[ai(k, l[a])], f[a][k]);
        }
        __syncthreads();
    }

    // wait for the earlier-coloured neighbours (np <= 64: first wavefront)
    if (tid < np) {
        const int32_t *fl = flags + preds[p0 + tid];
        dev::bounded_wait(fl, epoch, ctl, wait_ticks);
    }
    __syncthreads();

    // force += sums: device-scope loads (up to 8 per lane in flight), adds,
    // device-scope stores
    const __amdgpu_buffer_rsrc_t rf =
        __builtin_amdgcn_make_buffer_rsrc(d.force, 0, int32_t(24 * d.N), 0x00020000);
    auto foff = [&](int t, int k) {
        const int64_t g = s_id[t];
        return int32_t(8 * (LAYOUT == UM_AOS ? 3 * g + k : k * d.N + g));
    };
    constexpr int FB = 8;
    for (int u0 = tid; u0 < 3 * nn; u0 += FB * T) {
        double g[FB];
        int32_t off[FB], li[FB];
#pragma unroll
        for (int j = 0; j < FB; ++j) {
            const int u = u0 + j * T;
            const int t = LAYOUT == UM_AOS ? u / 3 : u % nn;
            const int k = LAYOUT == UM_AOS ? u % 3 : u / nn;
            li[j] = ai(k, t);
            off[j] = u < 3 * nn ? foff(t, k) : 0;
            g[j] = u < 3 * nn ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                              rf, off[j], 0, HEX_CPOL_SC1))
                              : 0.0;
        }
#pragma unroll
        for (int j = 0; j < FB; ++j)
            if (u0 + j * T < 3 * nn)
                __builtin_amdgcn_raw_buffer_store_b64(
                    __builtin_bit_cast(u32x2, g[j] + s_acc[li[j]]), rf, off[j], 0, HEX_CPOL_SC1);
    }
    // publish: every lane's stores complete, then one flag store
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + pos, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LAYOUT>
__device__ __forceinline__ void gather_element(const HexDats &d, const int32_t *row,
                                               double xe[8][3], double ve[8][3]) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        load3<LAYOUT>(d.x, d.N, row[a], xe[a]);
        load3<LAYOUT>(d.v, d.N, row[a], ve[a]);
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void hex_gcol_kernel(const int32_t *__restrict__ emap,
                                                       int32_t begin, int32_t end, HexDats d,
                                                       double kappa) {
    const int32_t s = begin + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= end) return;
    const int32_t *row = emap + 8 * int64_t(s);
    double xe[8][3], ve[8][3], f[8][3];
    gather_element<LAYOUT>(d, row, xe, ve);
    hex_force(xe, ve, kappa, f);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) d.force[idx3<LAYOUT>(d.N, row[a], k)] += f[a][k];
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void hex_atomic_kernel(const int32_t *__restrict__ emap,
                                                         int32_t n, HexDats d, double kappa) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int32_t *row = emap + 8 * int64_t(s);
    double xe[8][3], ve[8][3], f[8][3];
    gather_element<LAYOUT>(d, row, xe, ve);
    hex_force(xe, ve, kappa, f);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) unsafeAtomicAdd(&d.force[idx3<LAYOUT>(d.N, row[a], k)], f[a][k]);
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void hex_debug_kernel(const int32_t *__restrict__ emap,
                                                        int32_t n, HexDats d, double kappa,
                                                        double *__restrict__ out) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int32_t *row = emap + 8 * int64_t(s);
    double xe[8][3], ve[8][3], f[8][3];
    gather_element<LAYOUT>(d, row, xe, ve);
    hex_force_nocontract(xe, ve, kappa, f);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) out[24 * int64_t(s) + 3 * a + k] = f[a][k];
}

template <int LAYOUT>
hipError_t hex_launch_layout(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                             int64_t lds) {
    const HexDats d{static_cast<const double *>(la.x), static_cast<const double *>(la.q), la.res,
                    la.N};
    const double kappa = la.gm1;
    if (which == LAUNCH_HIER) {
        const bool atom = la.tcmode == UM_TC_LDS_ATOMIC;
        auto kern = atom ? hex_hier_kernel<LAYOUT, UM_TC_LDS_ATOMIC>
                         : hex_hier_kernel<LAYOUT, UM_TC_BARRIER>;
        clear_stale_error();
        const hipError_t ea = allow_lds(reinterpret_cast<const void *>(kern), lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(kern, dim3(end - begin), dim3(la.block_size), size_t(lds), la.stream,
                           la.binfo, la.stg_c, la.crun, reinterpret_cast<const uint4 *>(la.loc), d,
                           kappa, begin);
        return hipGetLastError();
    }
    if (which == LAUNCH_HIER_FLOW) {
        const bool atom = la.tcmode == UM_TC_LDS_ATOMIC;
        auto kern = atom ? hex_flow_kernel<LAYOUT, UM_TC_LDS_ATOMIC>
                         : hex_flow_kernel<LAYOUT, UM_TC_BARRIER>;
        clear_stale_error();
        const hipError_t ea = allow_lds(reinterpret_cast<const void *>(kern), lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(kern, dim3(end - begin), dim3(la.block_size), size_t(lds), la.stream,
                           la.binfo, la.stg_c, la.crun, reinterpret_cast<const uint4 *>(la.loc), d,
                           kappa, la.pred_off, la.preds, la.flags, la.err, la.wait_ticks);
        return hipGetLastError();
    }
    const int32_t n = end - begin;
    if (n <= 0) return hipSuccess;
    const int tb = la.block_size;
    dim3 grid((n + tb - 1) / tb), block(tb);
    clear_stale_error();
    if (which == LAUNCH_GCOL)
        hipLaunchKernelGGL((hex_gcol_kernel<LAYOUT>), grid, block, 0, la.stream, la.emap, begin,
                           end, d, kappa);
    else if (which == LAUNCH_ATOMIC)
        hipLaunchKernelGGL((hex_atomic_kernel<LAYOUT>), grid, block, 0, la.stream, la.emap, n, d,
                           kappa);
    else if (which == LAUNCH_DEBUG)
        hipLaunchKernelGGL((hex_debug_kernel<LAYOUT>), grid, block, 0, la.stream, la.emap, n, d,
                           kappa, la.out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t hex_launch_one(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                          int64_t lds) {
    return la.layout == UM_AOS ? hex_launch_layout<UM_AOS>(la, which, begin, end, lds)
                               : hex_launch_layout<UM_SOA>(la, which, begin, end, lds);
}

}  // namespace um
