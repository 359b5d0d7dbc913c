// gfx950 kernels of the 2D edge-flux indirect-increment loop.
//
//  hier_kernel   two-layer colouring (paper Section 2.2, Algorithm 1): one
//                workgroup per block.  The block's staged cells and nodes are
//                gathered into LDS (structure-of-arrays inside LDS), the
//                residuals of the staged cells are preloaded as the FP64
//                increment accumulators, every lane computes its edges'
//                fluxes into registers, increments are applied to LDS one
//                thread colour at a time with a workgroup barrier after each
//                colour, and the accumulators are stored back once.  Blocks
//                of one block colour write disjoint cells, so a launch per
//                block colour needs no atomics.
//  hier_flow_kernel  the same per-block work as one launch over all blocks
//                in colour order (dataflow schedule): a block's residual
//                read-modify-write waits for its earlier-coloured neighbours'
//                completion flags instead of a kernel boundary.
//  gcol_kernel   global colouring baseline (Section 2.1): one launch per
//                colour, gather through the int32 maps, plain read-modify-
//                write of res.
//  atomic_kernel atomics baseline (Section 2.1): one launch, hardware FP64
//                atomic adds on res.
//  debug_kernel  per-edge fluxes with floating-point contraction disabled.
//
// Every kernel is a template on the real type of x, q and adt (double, or
// float for the FP32-storage variant); the flux is evaluated in that type and
// the residual and its accumulators are always double.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "device_lf2d.hpp"
#include "device_staged.hpp"
#include "launch.hpp"

namespace um {
namespace {

using dev::lf2d_flux;
using dev::lf2d_flux_nocontract;
using dev::load2;
using dev::load4;
using dev::StagedIds;
using dev::store4;


// LDS floating-point add without return (ds_add_f64).  Inside one colour
// round no two lanes touch the same address, so the result equals a plain
// read-modify-write and stays deterministic; it is one LDS instruction
// instead of a read and a write.
__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename Real>
struct Dats {
    const Real *__restrict__ x;
    const Real *__restrict__ q;
    const Real *__restrict__ adt;
    double *__restrict__ res;
    int64_t N, C;
};

template <int LAYOUT, typename Real>
__device__ __forceinline__ void edge_flux_global(const Dats<Real> &d, int L, int R, int a, int b,
                                                 Real gm1, Real eps, Real f[4]) {
    Real qL[4], qR[4], xa0, xa1, xb0, xb1;
    load4<LAYOUT>(d.q, d.C, L, qL);
    load4<LAYOUT>(d.q, d.C, R, qR);
    load2<LAYOUT>(d.x, d.N, a, xa0, xa1);
    load2<LAYOUT>(d.x, d.N, b, xb0, xb1);
    const Real adtL = d.adt[L], adtR = d.adt[R];
    lf2d_flux(xa0, xa1, xb0, xb1, qL, qR, adtL, adtR, gm1, eps, f);
}

// One staged cell in registers between its global loads and LDS stores.
template <typename Real>
struct CellRegs {
    double r[4];
    Real q[4], a;
};

template <int LAYOUT, int STAGING, typename Real>
__device__ __forceinline__ void fetch_cell(const Dats<Real> &d, int64_t g, CellRegs<Real> &c) {
    load4<LAYOUT>(d.res, d.C, g, c.r);
    if constexpr (STAGING == UM_STAGE_ALL) {
        load4<LAYOUT>(d.q, d.C, g, c.q);
        c.a = d.adt[g];
    }
}

template <int STAGING, typename Real>
__device__ __forceinline__ void put_cell(double *s_inc, Real *s_q, Real *s_adt, int nc, int t,
                                         const CellRegs<Real> &c) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_inc[k * nc + t] = c.r[k];
    if constexpr (STAGING == UM_STAGE_ALL) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_q[k * nc + t] = c.q[k];
        s_adt[t] = c.a;
    }
}

// Colour code of an empty slot (padding of wave-pure colour groups).
constexpr int EMPTY_SLOT = 15;

// EPT = elements (edges) per lane: the workgroup has T lanes and handles a
// block of up to EPT*T edges; lane l computes slots l, l+T, ...
template <int LAYOUT, int STAGING, int TCMODE, int EPT, typename Real>
__global__ __launch_bounds__(1024) void hier_kernel(const BlockInfo *__restrict__ binfo,
                                                    const int32_t *__restrict__ stg_c,
                                                    const int32_t *__restrict__ stg_n,
                                                    const Run *__restrict__ crun,
                                                    const Run *__restrict__ nrun,
                                                    const uint32_t *__restrict__ loc,
                                                    int64_t n_slots, Dats<Real> d,
                                                    double gm1d, double epsd, int32_t base) {
    extern __shared__ double lds[];
    const Real gm1 = Real(gm1d), eps = Real(epsd);
    const int32_t pos = base + int32_t(blockIdx.x);
    const BlockInfo bi = binfo[pos], bn = binfo[pos + 1];
    const int ne = bn.slot_off - bi.slot_off;
    const int nc = bn.cell_off - bi.cell_off;
    const int nn = bn.node_off - bi.node_off;
    const int ncr = bn.crun_off - bi.crun_off, nnr = bn.nrun_off - bi.nrun_off;
    const int32_t *__restrict__ sc = stg_c + bi.cell_off;
    const int32_t *__restrict__ sn = stg_n + bi.node_off;
    StagedIds cell_id, node_id;
    cell_id.init(crun, bi.crun_off, ncr, sc);
    node_id.init(nrun, bi.nrun_off, nnr, sn);
    double *s_inc = lds;                                      // [4][nc] accumulators
    Real *s_q = reinterpret_cast<Real *>(s_inc + 4 * nc);     // [4][nc]
    Real *s_adt = s_q + 4 * nc;                               // [nc]
    Real *s_x = s_adt + nc;                                   // [2][nn]
    const int tid = int(threadIdx.x), T = int(blockDim.x);

    // local index words of this lane's slots: issued first, used after the
    // barrier
    const uint16_t *__restrict__ loc16 = reinterpret_cast<const uint16_t *>(loc + n_slots);
    uint32_t wa[EPT], wb[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int s = tid + j * T;
        wa[j] = s < ne ? loc[bi.slot_off + s] : 0u;
        wb[j] = s < ne ? uint32_t(loc16[bi.slot_off + s]) : 0u;
    }

    // gather: per pass every lane fetches at most one staged cell and one
    // staged node, issuing all their loads before any LDS store (one memory
    // wait per pass; a block of S edges usually has fewer than S staged
    // cells and nodes, so with one edge per lane a single pass covers it)
    const int npass = STAGING == UM_STAGE_ALL ? (nc > nn ? nc : nn) : nc;
    for (int t = tid; t < npass; t += T) {
        const bool hc = t < nc;
        const bool hn = STAGING == UM_STAGE_ALL && t < nn;
        // both ids before any load of the pass: an id read from an explicit
        // list after a data load would wait for that load
        const int32_t gc = hc ? cell_id(t) : 0;
        const int32_t gn = hn ? node_id(t) : 0;
        CellRegs<Real> c;
        Real xa = Real(0), xb = Real(0);
        if (hc) fetch_cell<LAYOUT, STAGING>(d, gc, c);
        if (hn) load2<LAYOUT>(d.x, d.N, gn, xa, xb);
        if (hc) put_cell<STAGING>(s_inc, s_q, s_adt, nc, t, c);
        if (hn) {
            s_x[t] = xa;
            s_x[nn + t] = xb;
        }
    }
    __syncthreads();

    // fluxes of this lane's edges into registers
    int lL[EPT], lR[EPT], col[EPT];
    Real f[EPT][4];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        lL[j] = int(wa[j] & 0x7FFu);
        lR[j] = int((wa[j] >> 11) & 0x7FFu);
        col[j] = (tid + j * T) < ne ? int(wb[j] >> 12) : -1;
        if (col[j] == EMPTY_SLOT) col[j] = -1;
        const int nA = int((wa[j] >> 22) | ((wb[j] & 1u) << 10));
        const int nB = int((wb[j] >> 1) & 0x7FFu);
#pragma unroll
        for (int k = 0; k < 4; ++k) f[j][k] = Real(0);
        if (col[j] >= 0) {
            if constexpr (STAGING == UM_STAGE_ALL) {
                Real qL[4], qR[4];
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
        // a cell, so their LDS updates do not race.  Slots are sorted by
        // colour, so most wavefronts hold a single colour.
        const int ncol = bi.ncol;
        for (int c = 0; c < ncol; ++c) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (col[j] == c) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        lds_add(&s_inc[k * nc + lL[j]], double(f[j][k]));
                        lds_add(&s_inc[k * nc + lR[j]], -double(f[j][k]));
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
                    lds_add(&s_inc[k * nc + lL[j]], double(f[j][k]));
                    lds_add(&s_inc[k * nc + lR[j]], -double(f[j][k]));
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

// Device-coherent residual accesses of the DATAFLOW schedule.  Blocks that
// hand residuals to each other may run on different XCDs, whose L2 caches
// are not coherent with each other.  A device-scope fence pair would make
// them coherent but writes back (release) and invalidates (acquire) the
// whole L2 of the XCD, once per block.  Instead every residual load and
// store of the schedule carries the device-scope cache policy (sc1) through
// a buffer resource covering res: stores write through to the device
// coherence point and loads do not return lines cached before, so only the
// order of completion has to be enforced (s_waitcnt before the flag store,
// the flag load before the residual loads).  The resource's record count is
// the byte size of res (at most 2^31 - 1, checked when the plan is built);
// an access outside it would be dropped by the hardware.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
constexpr int CPOL_SC1 = 16;  // device scope

__device__ __forceinline__ __amdgpu_buffer_rsrc_t res_rsrc(double *res, int64_t C) {
    return __builtin_amdgcn_make_buffer_rsrc(res, 0, int32_t(32 * C), 0x00020000);
}

template <int LAYOUT>
__device__ __forceinline__ void load4_dev(__amdgpu_buffer_rsrc_t r, int64_t C, int64_t g,
                                          double v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        const int32_t off = int32_t(32 * g);
        const f64x2 lo = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CPOL_SC1));
        const f64x2 hi = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, CPOL_SC1));
        v[0] = lo.x; v[1] = lo.y; v[2] = hi.x; v[3] = hi.y;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = __builtin_bit_cast(
                double, __builtin_amdgcn_raw_buffer_load_b64(r, int32_t(8 * (k * C + g)), 0, CPOL_SC1));
    }
}

template <int LAYOUT>
__device__ __forceinline__ void store4_dev(__amdgpu_buffer_rsrc_t r, int64_t C, int64_t g,
                                           const double v[4]) {
    if constexpr (LAYOUT == UM_AOS) {
        const int32_t off = int32_t(32 * g);
        const f64x2 lo = {v[0], v[1]}, hi = {v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, lo), r, off, 0, CPOL_SC1);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, hi), r, off + 16, 0, CPOL_SC1);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[k]), r,
                                                  int32_t(8 * (k * C + g)), 0, CPOL_SC1);
    }
}


// DATAFLOW schedule: one launch over all blocks in colour order (position =
// blockIdx.x).  Same per-block work as hier_kernel with STAGE_ALL and EPT
// edges per lane, except that the residuals are loaded only after every
// neighbouring block of an earlier colour has published its write-back (a
// first look at the flags goes out with the gathers; when all have already
// published, the residual loads overlap the flux evaluation, otherwise the
// block polls after it).
// Publication: all lanes finish their device-scope residual stores
// (s_waitcnt), the workgroup meets at a barrier, then one lane stores the
// execution's epoch into the block's flag (device-scope atomic store).
// Consumption: lanes of the first wavefront poll one predecessor flag each
// (device-scope atomic loads) until it holds the epoch; the barrier after
// the polls precedes the device-scope residual loads.  Blocks are dispatched in increasing
// blockIdx order and a block only waits for smaller positions, so every
// awaited block is already running or finished; the wait is bounded in time
// anyway (wait_ticks of s_memrealtime, 100 MHz) and a timeout is counted
// instead of hanging: ctl[0] counts timeouts, ctl[1] holds the epoch of the
// execution in which the last one happened, and the other waits of that
// same execution then give up at once (a later execution has a larger epoch
// and waits normally again).
// Execution numbers: a block's flag holds the number of executions it has
// completed, and every execution runs every block once, so all flags move
// in lockstep; a block's epoch is its own flag + 1 and a predecessor is done
// when its flag equals that epoch.  Nothing global is counted (a device-
// scope atomic per block on one shared counter serialises the whole launch)
// and a captured graph can replay the launch.
// Binary32 storage: asking for 8 waves per SIMD changes no register count
// (the kernel fits 64 VGPRs) but lets the compiler schedule for that
// occupancy, measured faster (FP32, two edges per lane: S = 512 71.4 ->
// 70.7 us, S = 1024 78.0 -> 71.4 us); the binary64 code is unchanged.
template <int LAYOUT, int TCMODE, int EPT, typename Real, bool SUM_FIRST>
__global__ __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 8 : 1))) void hier_flow_kernel(
    const BlockInfo *__restrict__ binfo, const int32_t *__restrict__ stg_c,
    const int32_t *__restrict__ stg_n, const Run *__restrict__ crun, const Run *__restrict__ nrun,
    const uint32_t *__restrict__ loc, int64_t n_slots, Dats<Real> d, double gm1d, double epsd,
    const int32_t *__restrict__ pred_off, const int32_t *__restrict__ preds, int32_t *flags,
    int32_t *ctl, uint64_t wait_ticks) {
    extern __shared__ double lds[];
    const int32_t pos = int32_t(blockIdx.x);
    const int32_t epoch =
        __hip_atomic_load(flags + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    const Real gm1 = Real(gm1d), eps = Real(epsd);
    const BlockInfo bi = binfo[pos], bn = binfo[pos + 1];
    const int ne = bn.slot_off - bi.slot_off;
    const int nc = bn.cell_off - bi.cell_off;
    const int nn = bn.node_off - bi.node_off;
    const int ncr = bn.crun_off - bi.crun_off, nnr = bn.nrun_off - bi.nrun_off;
    const int32_t *__restrict__ sc = stg_c + bi.cell_off;
    const int32_t *__restrict__ sn = stg_n + bi.node_off;
    StagedIds cell_id, node_id;
    cell_id.init(crun, bi.crun_off, ncr, sc);
    node_id.init(nrun, bi.nrun_off, nnr, sn);
    double *s_inc = lds;
    Real *s_q = reinterpret_cast<Real *>(s_inc + 4 * nc);
    Real *s_adt = s_q + 4 * nc;
    Real *s_x = s_adt + nc;
    const int tid = int(threadIdx.x), T = int(blockDim.x);
    const int p0 = pred_off[pos], np = pred_off[pos + 1] - p0;
    // a block likely to wait sums its fluxes from zero before its wait (a
    // plan without such blocks runs the instantiation without that path)
    const bool sum_first = SUM_FIRST && bi.sum_first != 0;
    if (sum_first)
        for (int u = tid; u < 4 * nc; u += T) s_inc[u] = 0.0;

    // local index words of this lane's slots tid, tid + T, ...
    const uint16_t *__restrict__ loc16 = reinterpret_cast<const uint16_t *>(loc + n_slots);
    uint32_t wa[EPT], wb[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int s = tid + j * T;
        wa[j] = s < ne ? loc[bi.slot_off + s] : 0u;
        wb[j] = s < ne ? uint32_t(loc16[bi.slot_off + s]) : 0u;
    }
    // one early look at the predecessors' flags, issued with the gathers: if
    // all of them have already published (the usual case, blocks are
    // launched in colour order), the residuals are loaded right after the
    // gather barrier and arrive while the fluxes are computed, instead of
    // after a wait at the end of the compute; the flag loads complete before
    // that barrier, so every residual load is issued after them
    __shared__ int s_ready;
    bool mine = true;
    if (tid < np)
        mine = __hip_atomic_load(flags + preds[p0 + tid], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) == epoch;
    const __amdgpu_buffer_rsrc_t rres = res_rsrc(d.res, d.C);
    // gather q, adt, x: each iteration issues the loads of EPT passes (one
    // staged cell and one staged node per lane and pass) before any LDS
    // store, so a block with more staged points than lanes still waits on
    // memory once per iteration
    const int npass = nc > nn ? nc : nn;
    int32_t gfirst[EPT];  // cell ids of the first pass, reused for the residuals
    for (int t0 = tid; t0 < npass; t0 += EPT * T) {
        Real qv[EPT][4], av[EPT], xa[EPT], xb[EPT];
        // all ids of the pass before any of its loads (an id read from an
        // explicit list after a data load would wait for that load)
        int32_t gc[EPT], gn[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int t = t0 + j * T;
            gc[j] = t < nc ? cell_id(t) : 0;
            gn[j] = t < nn ? node_id(t) : 0;
            if (t0 == tid) gfirst[j] = gc[j];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int t = t0 + j * T;
#pragma unroll
            for (int k = 0; k < 4; ++k) qv[j][k] = Real(0);
            av[j] = xa[j] = xb[j] = Real(0);
            if (t < nc) {
                load4<LAYOUT>(d.q, d.C, gc[j], qv[j]);
                av[j] = d.adt[gc[j]];
            }
            if (t < nn) load2<LAYOUT>(d.x, d.N, gn[j], xa[j], xb[j]);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int t = t0 + j * T;
            if (t < nc) {
#pragma unroll
                for (int k = 0; k < 4; ++k) s_q[k * nc + t] = qv[j][k];
                s_adt[t] = av[j];
            }
            if (t < nn) {
                s_x[t] = xa[j];
                s_x[nn + t] = xb[j];
            }
        }
    }
    if (tid < 64) {  // np <= 64: the flags are all in the first wavefront
        const bool all = __all(mine);
        if (tid == 0) s_ready = all ? 1 : 0;
    }
    __syncthreads();
    const bool ready = s_ready != 0;
    double r0[EPT][4];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
#pragma unroll
        for (int k = 0; k < 4; ++k) r0[j][k] = 0.0;
        if (ready && !sum_first && tid + j * T < nc) load4_dev<LAYOUT>(rres, d.C, gfirst[j], r0[j]);
    }

    // fluxes of this lane's edges into registers
    int lL[EPT], lR[EPT], col[EPT];
    Real f[EPT][4];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        lL[j] = int(wa[j] & 0x7FFu);
        lR[j] = int((wa[j] >> 11) & 0x7FFu);
        col[j] = (tid + j * T) < ne ? int(wb[j] >> 12) : -1;
        if (col[j] == EMPTY_SLOT) col[j] = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) f[j][k] = Real(0);
        if (col[j] >= 0) {
            const int nA = int((wa[j] >> 22) | ((wb[j] & 1u) << 10));
            const int nB = int((wb[j] >> 1) & 0x7FFu);
            Real qL[4], qR[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                qL[k] = s_q[k * nc + lL[j]];
                qR[k] = s_q[k * nc + lR[j]];
            }
            lf2d_flux(s_x[nA], s_x[nn + nA], s_x[nB], s_x[nn + nB], qL, qR, s_adt[lL[j]],
                      s_adt[lR[j]], gm1, eps, f[j]);
        }
    }

    if (sum_first) {
        // the accumulators were zeroed before the gather barrier
    } else if (ready) {  // uniform over the block
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int t = tid + j * T;
            if (t < nc) {
#pragma unroll
                for (int k = 0; k < 4; ++k) s_inc[k * nc + t] = r0[j][k];
            }
        }
        for (int t = tid + EPT * T; t < nc; t += T) {
            double r[4];
            load4_dev<LAYOUT>(rres, d.C, cell_id(t), r);
#pragma unroll
            for (int k = 0; k < 4; ++k) s_inc[k * nc + t] = r[k];
        }
        __syncthreads();
    } else {
        // wait for the earlier-coloured neighbours
        if (tid < np) {
            const int32_t *fl = flags + preds[p0 + tid];
            dev::bounded_wait(fl, epoch, ctl, wait_ticks);
        }
        __syncthreads();
        // residuals as accumulators
        for (int t = tid; t < nc; t += T) {
            double r[4];
            load4_dev<LAYOUT>(rres, d.C, cell_id(t), r);
#pragma unroll
            for (int k = 0; k < 4; ++k) s_inc[k * nc + t] = r[k];
        }
        __syncthreads();
    }

    if constexpr (TCMODE == UM_TC_BARRIER) {
        const int ncol = bi.ncol;
        for (int c = 0; c < ncol; ++c) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (col[j] == c) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        lds_add(&s_inc[k * nc + lL[j]], double(f[j][k]));
                        lds_add(&s_inc[k * nc + lR[j]], -double(f[j][k]));
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
                    lds_add(&s_inc[k * nc + lL[j]], double(f[j][k]));
                    lds_add(&s_inc[k * nc + lR[j]], -double(f[j][k]));
                }
            }
        }
        __syncthreads();
    }

    if (sum_first) {
        // wait for the earlier-coloured neighbours, then res += sums
        if (tid < np) {
            const int32_t *fl = flags + preds[p0 + tid];
            dev::bounded_wait(fl, epoch, ctl, wait_ticks);
        }
        __syncthreads();
        for (int t = tid; t < nc; t += T) {
            const int32_t g = cell_id(t);
            double r[4];
            load4_dev<LAYOUT>(rres, d.C, g, r);
#pragma unroll
            for (int k = 0; k < 4; ++k) r[k] += s_inc[k * nc + t];
            store4_dev<LAYOUT>(rres, d.C, g, r);
        }
    } else {
        if constexpr (LAYOUT == UM_AOS) {
            // write-through stores: lane pairs write the two 16-byte halves of a
            // cell, so that one store instruction covers whole lines of a run of
            // consecutive cells (a partly written line costs a second write)
            for (int u = tid; u < 2 * nc; u += T) {
                const int t = u >> 1, h = u & 1;
                const f64x2 v = {s_inc[(2 * h) * nc + t], s_inc[(2 * h + 1) * nc + t]};
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rres,
                                                       int32_t(32 * int64_t(cell_id(t)) + 16 * h), 0,
                                                       CPOL_SC1);
            }
        } else {
            for (int t = tid; t < nc; t += T) {
                double r[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) r[k] = s_inc[k * nc + t];
                store4_dev<LAYOUT>(rres, d.C, cell_id(t), r);
            }
        }
    }
    // publish: every lane's stores complete, then one flag store
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + pos, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// DATAFLOW schedule with the gather done by LDS DMA (UM_GATHER_LDS_DMA, AoS
// data): the loads of the staged q, adt, x and residuals write LDS directly
// (buffer loads with the LDS bit: lane i of a wavefront lands at the
// wavefront's LDS base + i * size), so no registers hold staged data.  The
// block's order of work:
//   1. scalar loads of its 256-byte record (FlowRec): ranges, counts,
//      predecessors and the run descriptors of its staged lists;
//   2. one round trip: its own flag (its epoch), the predecessors' flags
//      (every wavefront reads them itself), this lane's local index words,
//      and the DMA of q, adt and x of the staged points (addresses from the
//      run descriptors in scalar registers; a block with an explicit list
//      loads its ids first);
//   3. a wavefront that saw every predecessor published issues the DMA of
//      its cells' residuals, then every lane evaluates its fluxes from LDS
//      while those arrive; a wavefront that was not ready polls its
//      predecessors (bounded wait) after its fluxes and fetches then;
//   4. thread-colour rounds into the residual accumulators, write-back with
//      device-scope stores, completion flag (as hier_flow_kernel).
// A block whose record says sum_first (its latest awaited neighbour was
// launched so shortly before it that it is likely still running) instead
// zeroes the accumulators, runs the rounds on them, then waits, then adds
// them to its cells' residuals with device-scope loads and stores: a chain
// of such blocks carries only that read-add-write between neighbours.
// LDS layout (each staged record split so that every DMA lands in 16-byte
// lanes): residual accumulators as two arrays of (res0, res1) and (res2, res3)
// pairs, then q (binary64: two arrays of pairs; binary32: one float4 array),
// x (binary64: one array of pairs; binary32: two arrays of words), adt
// (binary64: low and high words; binary32: one array).
typedef __attribute__((address_space(3))) void lds_void_t;

// (the builtin takes its size and cache policy as literal constants)
template <int SIZE, int CPOL = 0>
__device__ __forceinline__ void dma(__amdgpu_buffer_rsrc_t r, void *lds_wave_base, int32_t voff) {
    static_assert((SIZE == 4 || SIZE == 16) && (CPOL == 0 || CPOL == CPOL_SC1));
    lds_void_t *l = (lds_void_t *)lds_wave_base;
    if constexpr (SIZE == 16 && CPOL == 0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, l, 16, voff, 0, 0, 0);
    else if constexpr (SIZE == 16)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, l, 16, voff, 0, 0, 16);
    else if constexpr (CPOL == 0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, l, 4, voff, 0, 0, 0);
    else
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, l, 4, voff, 0, 0, 16);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, int32_t(bytes), 0x00020000);
}

// Id at staged position t from the record's run descriptors (scalar
// registers); nr >= 1.
__device__ __forceinline__ int32_t run_id(const Run (&runs)[MAX_RUNS], int32_t nr, int t) {
    int32_t g = runs[0].start + t;
#pragma unroll
    for (int r = 1; r < MAX_RUNS; ++r)
        if (r < nr && t >= runs[r].local) g = runs[r].start + (t - runs[r].local);
    return g;
}

// Id at staged position t: from the runs, or from the explicit list when the
// record has none.  The kernel calls the list form only on code paths of
// blocks with an explicit list: a load on a path merged with the DMA issue
// would make every later DMA wait for all earlier ones.
__device__ __forceinline__ int32_t rec_id(const Run (&runs)[MAX_RUNS], int32_t nr,
                                          const int32_t *__restrict__ list, int t) {
    return nr == 0 ? list[t] : run_id(runs, nr, t);
}

template <int TCMODE, int EPT, typename Real, bool SUM_FIRST>
__global__ __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 8 : 1))) void hier_dma_kernel(
    const FlowRec *__restrict__ frec, const int32_t *__restrict__ stg_c,
    const int32_t *__restrict__ stg_n, const uint32_t *__restrict__ loc, int64_t n_slots,
    Dats<Real> d, double gm1d, double epsd, const int32_t *__restrict__ preds, int32_t *flags,
    int32_t *ctl, uint64_t wait_ticks) {
    constexpr bool F64 = sizeof(Real) == 8;
    extern __shared__ double lds[];
    const int32_t pos = int32_t(blockIdx.x);
    const Real gm1 = Real(gm1d), eps = Real(epsd);
    // ---- 1. the block's record (uniform: scalar loads)
    const FlowRec &rec = frec[pos];
    const int ne = rec.ne, nc = rec.nc, nn = rec.nn, np = rec.np;
    const int ncr = rec.ncr, nnr = rec.nnr;
    // a plan without sum-first blocks runs the instantiation without that path
    const bool sum_first = SUM_FIRST && rec.sum_first != 0;
    Run cruns[MAX_RUNS], nruns[MAX_RUNS];
#pragma unroll
    for (int k = 0; k < MAX_RUNS; ++k) {
        cruns[k] = rec.cruns[k];
        nruns[k] = rec.nruns[k];
    }
    const int32_t *__restrict__ clist = stg_c + rec.cell_off;
    const int32_t *__restrict__ nlist = stg_n + rec.node_off;
    const int tid = int(threadIdx.x), T = int(blockDim.x), lane = tid & 63;

    // ---- 2. flags, local index words and the gather, one round trip.  No
    // value of these loads is used before every one of them is issued: a
    // use makes the wavefront wait for all loads issued before it.
    int32_t ep0 = __hip_atomic_load(flags + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t pf;
    if (np <= 8) {
        // predecessors from scalar registers (selecting values, not
        // addresses: the selected address would be a vector load to wait for)
        int32_t pk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            pk[k] = rec.preds[k];
            asm volatile("" : "+s"(pk[k]));
        }
        int32_t pr = pos;
#pragma unroll
        for (int k = 0; k < 8; ++k) pr = lane == k && k < np ? pk[k] : pr;
        pf = __hip_atomic_load(flags + pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const int32_t pr = lane < np ? preds[rec.p0 + lane] : pos;
        pf = __hip_atomic_load(flags + pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint16_t *__restrict__ loc16 = reinterpret_cast<const uint16_t *>(loc + n_slots);
    uint32_t wa[EPT], wb[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int s = tid + j * T;
        wa[j] = s < ne ? loc[rec.slot_off + s] : 0u;
        wb[j] = s < ne ? uint32_t(loc16[rec.slot_off + s]) : 0u;
    }

    // LDS regions
    double *r_lo = lds;                 // [nc] x (res0, res1)
    double *r_hi = r_lo + 2 * nc;       // [nc] x (res2, res3)
    Real *q_a = reinterpret_cast<Real *>(r_hi + 2 * nc);  // F64: [nc] x (q0, q1); F32: [nc] x q[4]
    Real *q_b = q_a + 2 * nc;           // F64: [nc] x (q2, q3)
    Real *x_a = q_a + 4 * nc;           // F64: [nn] x (x, y); F32: [nn] x
    Real *x_b = x_a + nn;               // F32: [nn] y
    uint32_t *adt_w = reinterpret_cast<uint32_t *>(x_a + 2 * nn);  // F64: [2][nc] words; F32: [nc]
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(d.q, 4 * sizeof(Real) * d.C);
    const __amdgpu_buffer_rsrc_t ra = rsrc_of(d.adt, sizeof(Real) * d.C);
    const __amdgpu_buffer_rsrc_t rx = rsrc_of(d.x, 2 * sizeof(Real) * d.N);
    const __amdgpu_buffer_rsrc_t rres = res_rsrc(d.res, d.C);

    auto cell_dma = [&](int t0, int32_t g) {
        if constexpr (F64) {
            dma<16>(rq, q_a + 2 * t0, 32 * g);
            dma<16>(rq, q_b + 2 * t0, 32 * g + 16);
            dma<4>(ra, adt_w + t0, 8 * g);
            dma<4>(ra, adt_w + nc + t0, 8 * g + 4);
        } else {
            dma<16>(rq, q_a + 4 * t0, 16 * g);
            dma<4>(ra, adt_w + t0, 4 * g);
        }
    };
    auto node_dma = [&](int t0, int32_t g) {
        if constexpr (F64) {
            dma<16>(rx, x_a + 2 * t0, 16 * g);
        } else {
            dma<4>(rx, x_a + t0, 8 * g);
            dma<4>(rx, x_b + t0, 8 * g + 4);
        }
    };
    const int npass = nc > nn ? nc : nn;
    const int tw = __builtin_amdgcn_readfirstlane(tid - lane);  // first position of the wave
    if (ncr > 0 && nnr > 0) {
        // both lists as runs: addresses from scalar registers, no loads
        for (int t0 = tw; t0 < npass; t0 += T) {
            const int t = t0 + lane;
            if (t < nc) cell_dma(t0, run_id(cruns, ncr, t));
            if (t < nn) node_dma(t0, run_id(nruns, nnr, t));
        }
    } else {
        // an explicit list: each pass loads its ids, then issues its DMAs
        for (int t0 = tw; t0 < npass; t0 += T) {
            const int t = t0 + lane;
            const int32_t gc = t < nc ? rec_id(cruns, ncr, clist, t) : 0;
            const int32_t gn = t < nn ? rec_id(nruns, nnr, nlist, t) : 0;
            if (t < nc) cell_dma(t0, gc);
            if (t < nn) node_dma(t0, gn);
        }
    }
    asm volatile("" : "+v"(ep0), "+v"(pf));  // every load above is issued by now
    const int32_t epoch = ep0 + 1;
    const bool ready = __all(lane >= np || pf == epoch);  // this wavefront's view
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- 3. residuals of the ready wavefronts in flight during the fluxes
    auto fetch_res = [&]() {
        auto res_dma = [&](int t0, int32_t g) {
            dma<16, CPOL_SC1>(rres, r_lo + 2 * t0, 32 * g);
            dma<16, CPOL_SC1>(rres, r_hi + 2 * t0, 32 * g + 16);
        };
        if (ncr > 0) {
            for (int t0 = tw; t0 < nc; t0 += T)
                if (t0 + lane < nc) res_dma(t0, run_id(cruns, ncr, t0 + lane));
        } else {
            for (int t0 = tw; t0 < nc; t0 += T) {
                const int t = t0 + lane;
                const int32_t g = t < nc ? clist[t] : 0;
                if (t < nc) res_dma(t0, g);
            }
        }
    };
    if (sum_first) {
        for (int u = tid; u < 4 * nc; u += T) lds[u] = 0.0;
    } else if (ready) {
        fetch_res();
    }

    int lL[EPT], lR[EPT], col[EPT];
    Real f[EPT][4];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        lL[j] = int(wa[j] & 0x7FFu);
        lR[j] = int((wa[j] >> 11) & 0x7FFu);
        col[j] = (tid + j * T) < ne ? int(wb[j] >> 12) : -1;
        if (col[j] == EMPTY_SLOT) col[j] = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) f[j][k] = Real(0);
        if (col[j] >= 0) {
            const int nA = int((wa[j] >> 22) | ((wb[j] & 1u) << 10));
            const int nB = int((wb[j] >> 1) & 0x7FFu);
            Real qL[4], qR[4], aL, aR, xa0, xa1, xb0, xb1;
            if constexpr (F64) {
                const f64x2 l0 = *reinterpret_cast<const f64x2 *>(q_a + 2 * lL[j]);
                const f64x2 l1 = *reinterpret_cast<const f64x2 *>(q_b + 2 * lL[j]);
                const f64x2 r0 = *reinterpret_cast<const f64x2 *>(q_a + 2 * lR[j]);
                const f64x2 r1 = *reinterpret_cast<const f64x2 *>(q_b + 2 * lR[j]);
                qL[0] = l0.x; qL[1] = l0.y; qL[2] = l1.x; qL[3] = l1.y;
                qR[0] = r0.x; qR[1] = r0.y; qR[2] = r1.x; qR[3] = r1.y;
                aL = __builtin_bit_cast(double, uint64_t(adt_w[lL[j]]) |
                                                    (uint64_t(adt_w[nc + lL[j]]) << 32));
                aR = __builtin_bit_cast(double, uint64_t(adt_w[lR[j]]) |
                                                    (uint64_t(adt_w[nc + lR[j]]) << 32));
                const f64x2 xa = *reinterpret_cast<const f64x2 *>(x_a + 2 * nA);
                const f64x2 xb = *reinterpret_cast<const f64x2 *>(x_a + 2 * nB);
                xa0 = xa.x; xa1 = xa.y; xb0 = xb.x; xb1 = xb.y;
            } else {
                const float4 l = *reinterpret_cast<const float4 *>(q_a + 4 * lL[j]);
                const float4 r = *reinterpret_cast<const float4 *>(q_a + 4 * lR[j]);
                qL[0] = l.x; qL[1] = l.y; qL[2] = l.z; qL[3] = l.w;
                qR[0] = r.x; qR[1] = r.y; qR[2] = r.z; qR[3] = r.w;
                aL = __builtin_bit_cast(float, adt_w[lL[j]]);
                aR = __builtin_bit_cast(float, adt_w[lR[j]]);
                xa0 = x_a[nA]; xa1 = x_b[nA]; xb0 = x_a[nB]; xb1 = x_b[nB];
            }
            lf2d_flux(xa0, xa1, xb0, xb1, qL, qR, aL, aR, gm1, eps, f[j]);
        }
    }
    if (!ready && !sum_first) {
        // this wavefront waits for the earlier-coloured neighbours now
        if (lane < np) {
            int32_t pr = rec.preds[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) pr = lane == k ? rec.preds[k] : pr;
            if (np > 8) pr = preds[rec.p0 + lane];
            dev::bounded_wait(flags + pr, epoch, ctl, wait_ticks);
        }
        fetch_res();
    }
    // the fluxes are complete before the wait for the residual DMA (an
    // empty asm statement per value orders them before the s_waitcnt)
#pragma unroll
    for (int j = 0; j < EPT; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" ::"v"(f[j][k]));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- 4. thread-colour rounds into the accumulators
    auto acc = [&](int l, int k) -> double * { return (k < 2 ? r_lo : r_hi) + 2 * l + (k & 1); };
    if constexpr (TCMODE == UM_TC_BARRIER) {
        const int ncol = rec.ncol;
        for (int c = 0; c < ncol; ++c) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (col[j] == c) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        lds_add(acc(lL[j], k), double(f[j][k]));
                        lds_add(acc(lR[j], k), -double(f[j][k]));
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
                    lds_add(acc(lL[j], k), double(f[j][k]));
                    lds_add(acc(lR[j], k), -double(f[j][k]));
                }
            }
        }
        __syncthreads();
    }

    if (sum_first) {
        // wait for the earlier-coloured neighbours, then res += sums, lane
        // pairs on the two 16-byte halves of a cell, 4 halves per lane in flight
        if (tid < np) {
            int32_t pr = rec.preds[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) pr = lane == k ? rec.preds[k] : pr;
            if (np > 8) pr = preds[rec.p0 + lane];
            dev::bounded_wait(flags + pr, epoch, ctl, wait_ticks);
        }
        __syncthreads();
        for (int u0 = tid; u0 < 2 * nc; u0 += 4 * T) {
            int32_t off[4];
            f64x2 a[4];
            u32x4 v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = u0 + i * T < 2 * nc ? u0 + i * T : 0;
                const int32_t g = rec_id(cruns, ncr, clist, u >> 1);
                off[i] = int32_t(32 * int64_t(g) + 16 * (u & 1));
                a[i] = *reinterpret_cast<const f64x2 *>(((u & 1) ? r_hi : r_lo) + 2 * (u >> 1));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                v[i] = u0 + i * T < 2 * nc
                           ? __builtin_amdgcn_raw_buffer_load_b128(rres, off[i], 0, CPOL_SC1)
                           : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (u0 + i * T < 2 * nc) {
                    f64x2 r = __builtin_bit_cast(f64x2, v[i]);
                    r.x += a[i].x;
                    r.y += a[i].y;
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, r), rres,
                                                           off[i], 0, CPOL_SC1);
                }
            }
        }
    } else {
        // ---- write-back: lane pairs store the two 16-byte halves of a cell
        auto store_half = [&](int t, int h, int32_t g) {
            const f64x2 v = *reinterpret_cast<const f64x2 *>((h ? r_hi : r_lo) + 2 * t);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rres,
                                                   int32_t(32 * int64_t(g) + 16 * h), 0, CPOL_SC1);
        };
        if (ncr > 0) {
            for (int u = tid; u < 2 * nc; u += T) store_half(u >> 1, u & 1, run_id(cruns, ncr, u >> 1));
        } else {
            // the ids of all this lane's cells first (a list load after a store
            // would wait for the store)
            int32_t g[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = tid + i * T;
                g[i] = u < 2 * nc ? clist[u >> 1] : 0;
            }
            for (int u = tid, i = 0; u < 2 * nc; u += T, ++i) {
                const int32_t gi = i < 4 ? g[i] : clist[u >> 1];
                store_half(u >> 1, u & 1, gi);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + pos, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void gcol_kernel(const int4 *__restrict__ emap, int32_t begin,
                                                   int32_t end, Dats<Real> d, double gm1,
                                                   double eps) {
    const int32_t s = begin + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= end) return;
    const int4 m = emap[s];  // L, R, a, b
    Real f[4];
    edge_flux_global<LAYOUT>(d, m.x, m.y, m.z, m.w, Real(gm1), Real(eps), f);
    double rL[4], rR[4];
    load4<LAYOUT>(d.res, d.C, m.x, rL);
    load4<LAYOUT>(d.res, d.C, m.y, rR);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        rL[k] += double(f[k]);
        rR[k] -= double(f[k]);
    }
    store4<LAYOUT>(d.res, d.C, m.x, rL);
    store4<LAYOUT>(d.res, d.C, m.y, rR);
}

template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void atomic_kernel(const int4 *__restrict__ emap, int32_t n,
                                                     Dats<Real> d, double gm1, double eps) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int4 m = emap[s];
    Real f[4];
    edge_flux_global<LAYOUT>(d, m.x, m.y, m.z, m.w, Real(gm1), Real(eps), f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t iL = LAYOUT == UM_AOS ? 4 * int64_t(m.x) + k : k * d.C + m.x;
        const int64_t iR = LAYOUT == UM_AOS ? 4 * int64_t(m.y) + k : k * d.C + m.y;
        unsafeAtomicAdd(&d.res[iL], double(f[k]));
        unsafeAtomicAdd(&d.res[iR], -double(f[k]));
    }
}

template <int LAYOUT, typename Real>
__global__ __launch_bounds__(1024) void debug_kernel(const int4 *__restrict__ emap, int32_t n,
                                                    Dats<Real> d, double gm1, double eps,
                                                    double *__restrict__ out) {
    const int32_t s = int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= n) return;
    const int4 m = emap[s];
    Real qL[4], qR[4], xa0, xa1, xb0, xb1, f[4];
    load4<LAYOUT>(d.q, d.C, m.x, qL);
    load4<LAYOUT>(d.q, d.C, m.y, qR);
    load2<LAYOUT>(d.x, d.N, m.z, xa0, xa1);
    load2<LAYOUT>(d.x, d.N, m.w, xb0, xb1);
    lf2d_flux_nocontract(xa0, xa1, xb0, xb1, qL, qR, d.adt[m.x], d.adt[m.y], Real(gm1), Real(eps),
                         f);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * int64_t(s) + k] = double(f[k]);
}

template <int LAYOUT, int ST, int TC, int EPT, typename Real>
hipError_t launch_hier_one(const LaunchArgs &la, int32_t nblocks, int32_t base, int64_t lds,
                           const Dats<Real> &d) {
    clear_stale_error();
    const hipError_t ea =
        allow_lds(reinterpret_cast<const void *>(hier_kernel<LAYOUT, ST, TC, EPT, Real>), lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((hier_kernel<LAYOUT, ST, TC, EPT, Real>), dim3(nblocks),
                       dim3(la.block_size), size_t(lds), la.stream, la.binfo, la.stg_c, la.stg_n,
                       la.crun, la.nrun, la.loc, la.n_slots, d, la.gm1,
                       la.eps, base);
    return hipGetLastError();
}

template <int LAYOUT, int ST, int TC, typename Real>
hipError_t launch_hier_ept(const LaunchArgs &la, int32_t nblocks, int32_t base, int64_t lds,
                           const Dats<Real> &d) {
    if (la.ept == 1) return launch_hier_one<LAYOUT, ST, TC, 1>(la, nblocks, base, lds, d);
    if (la.ept == 2) return launch_hier_one<LAYOUT, ST, TC, 2>(la, nblocks, base, lds, d);
    return hipErrorInvalidValue;
}

template <int LAYOUT, typename Real>
hipError_t launch_hier(const LaunchArgs &la, int32_t nblocks, int32_t base, int64_t lds,
                       const Dats<Real> &d) {
    if (la.staging == UM_STAGE_ALL && la.tcmode == UM_TC_BARRIER)
        return launch_hier_ept<LAYOUT, UM_STAGE_ALL, UM_TC_BARRIER>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_ALL && la.tcmode == UM_TC_LDS_ATOMIC)
        return launch_hier_ept<LAYOUT, UM_STAGE_ALL, UM_TC_LDS_ATOMIC>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_INC_ONLY && la.tcmode == UM_TC_BARRIER)
        return launch_hier_ept<LAYOUT, UM_STAGE_INC_ONLY, UM_TC_BARRIER>(la, nblocks, base, lds, d);
    if (la.staging == UM_STAGE_INC_ONLY && la.tcmode == UM_TC_LDS_ATOMIC)
        return launch_hier_ept<LAYOUT, UM_STAGE_INC_ONLY, UM_TC_LDS_ATOMIC>(la, nblocks, base, lds,
                                                                            d);
    return hipErrorInvalidValue;
}

template <int LAYOUT, int TC, int EPT, typename Real, bool SF>
hipError_t launch_flow_sf(const LaunchArgs &la, int32_t nblocks, int64_t lds,
                          const Dats<Real> &d) {
    clear_stale_error();
    const hipError_t ea = allow_lds(
        reinterpret_cast<const void *>(hier_flow_kernel<LAYOUT, TC, EPT, Real, SF>), lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((hier_flow_kernel<LAYOUT, TC, EPT, Real, SF>), dim3(nblocks),
                       dim3(la.block_size), size_t(lds), la.stream, la.binfo, la.stg_c, la.stg_n,
                       la.crun, la.nrun, la.loc, la.n_slots, d, la.gm1, la.eps, la.pred_off,
                       la.preds, la.flags, la.err, la.wait_ticks);
    return hipGetLastError();
}

template <int LAYOUT, int TC, int EPT, typename Real>
hipError_t launch_flow_one(const LaunchArgs &la, int32_t nblocks, int64_t lds,
                           const Dats<Real> &d) {
    return la.sum_first ? launch_flow_sf<LAYOUT, TC, EPT, Real, true>(la, nblocks, lds, d)
                        : launch_flow_sf<LAYOUT, TC, EPT, Real, false>(la, nblocks, lds, d);
}

template <int TC, int EPT, typename Real, bool SF>
hipError_t launch_dma_sf(const LaunchArgs &la, int32_t nblocks, int64_t lds,
                         const Dats<Real> &d) {
    clear_stale_error();
    const hipError_t ea =
        allow_lds(reinterpret_cast<const void *>(hier_dma_kernel<TC, EPT, Real, SF>), lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((hier_dma_kernel<TC, EPT, Real, SF>), dim3(nblocks), dim3(la.block_size),
                       size_t(lds), la.stream, la.frec, la.stg_c, la.stg_n, la.loc, la.n_slots, d,
                       la.gm1, la.eps, la.preds, la.flags, la.err, la.wait_ticks);
    return hipGetLastError();
}

template <int TC, int EPT, typename Real>
hipError_t launch_dma_one(const LaunchArgs &la, int32_t nblocks, int64_t lds,
                          const Dats<Real> &d) {
    return la.sum_first ? launch_dma_sf<TC, EPT, Real, true>(la, nblocks, lds, d)
                        : launch_dma_sf<TC, EPT, Real, false>(la, nblocks, lds, d);
}

template <int LAYOUT, int TC, typename Real>
hipError_t launch_flow(const LaunchArgs &la, int32_t nblocks, int64_t lds, const Dats<Real> &d) {
    if (la.gather == UM_GATHER_LDS_DMA) {
        if constexpr (LAYOUT == UM_AOS) {
            if (la.ept == 1) return launch_dma_one<TC, 1>(la, nblocks, lds, d);
            if (la.ept == 2) return launch_dma_one<TC, 2>(la, nblocks, lds, d);
        }
        return hipErrorInvalidValue;
    }
    if (la.ept == 1) return launch_flow_one<LAYOUT, TC, 1>(la, nblocks, lds, d);
    if (la.ept == 2) return launch_flow_one<LAYOUT, TC, 2>(la, nblocks, lds, d);
    return hipErrorInvalidValue;
}

template <int LAYOUT, typename Real>
hipError_t launch_typed(const LaunchArgs &la, int which, int32_t begin, int32_t end, int64_t lds) {
    const Dats<Real> d{static_cast<const Real *>(la.x), static_cast<const Real *>(la.q),
                       static_cast<const Real *>(la.adt), la.res, la.N, la.C};
    if (which == LAUNCH_HIER) return launch_hier<LAYOUT>(la, end - begin, begin, lds, d);
    if (which == LAUNCH_HIER_FLOW) {
        if (la.staging != UM_STAGE_ALL || (la.ept != 1 && la.ept != 2) || end - begin <= 0)
            return hipErrorInvalidValue;
        return la.tcmode == UM_TC_BARRIER
                   ? launch_flow<LAYOUT, UM_TC_BARRIER>(la, end - begin, lds, d)
                   : launch_flow<LAYOUT, UM_TC_LDS_ATOMIC>(la, end - begin, lds, d);
    }
    const int32_t n = end - begin;
    if (n <= 0) return hipSuccess;
    const int tb = la.block_size;
    dim3 grid((n + tb - 1) / tb), block(tb);
    const int4 *em = reinterpret_cast<const int4 *>(la.emap);
    clear_stale_error();
    if (which == LAUNCH_GCOL)
        hipLaunchKernelGGL((gcol_kernel<LAYOUT, Real>), grid, block, 0, la.stream, em, begin, end,
                           d, la.gm1, la.eps);
    else if (which == LAUNCH_ATOMIC)
        hipLaunchKernelGGL((atomic_kernel<LAYOUT, Real>), grid, block, 0, la.stream, em, n, d,
                           la.gm1, la.eps);
    else if (which == LAUNCH_DEBUG)
        hipLaunchKernelGGL((debug_kernel<LAYOUT, Real>), grid, block, 0, la.stream, em, n, d,
                           la.gm1, la.eps, la.out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t lf2d_launch_one(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                           int64_t lds) {
    const bool f64 = la.dtype == UM_F64;
    if (la.layout == UM_AOS)
        return f64 ? launch_typed<UM_AOS, double>(la, which, begin, end, lds)
                   : launch_typed<UM_AOS, float>(la, which, begin, end, lds);
    return f64 ? launch_typed<UM_SOA, double>(la, which, begin, end, lds)
               : launch_typed<UM_SOA, float>(la, which, begin, end, lds);
}

}  // namespace um
