// Launch descriptors shared by the ABI layer and the HIP kernel files.
#pragma once

#include <hip/hip_runtime_api.h>

#include <mutex>
#include <set>
#include <utility>

#include "internal.hpp"

namespace um {

enum { LAUNCH_HIER = 0, LAUNCH_GCOL = 1, LAUNCH_ATOMIC = 2, LAUNCH_DEBUG = 3,
       LAUNCH_HIER_FLOW = 4, LAUNCH_DIRECT = 5, LAUNCH_REDUCE = 6 };

struct LaunchArgs {
    hipStream_t stream;
    int32_t layout, staging, tcmode, block_size, ept, dtype;
    const BlockInfo *binfo;
    const int32_t *stg_c, *stg_n;
    const Run *crun, *nrun;
    const uint32_t *loc;
    int64_t n_slots;          // LF2D: slots of the plan (the 16-bit halves follow the words)
    const int32_t *emap;
    const void *x, *q, *adt;  // UM_F64 or UM_F32 per dtype
    double *res;
    int64_t N, C;
    double gm1, eps;
    double *out;  // debug fluxes
    int32_t schedule;
    const int32_t *pred_off, *preds;
    const FlowRec *frec;      // DATAFLOW edge loop: per launch position
    int32_t gather;           // HIER, DATAFLOW: um_gather
    int32_t sum_first;        // DATAFLOW edge loop: 1 if any block sums before its wait
    int32_t *flags, *err;  // DATAFLOW: completion flags; err = control words [4]
    uint64_t wait_ticks;   // DATAFLOW: longest wait for one neighbour (100 MHz ticks)
    double qinf[4];        // BOUNDARY_FLUX: far-field state
    double *partials;      // UPDATE: per-workgroup sums
    double *gbl;           // UPDATE: the global reduction target
    int32_t n_partials;
};

// Clears an error left in the thread's HIP state by an earlier, unrelated
// runtime call, so that hipGetLastError() after a launch reports that
// launch only.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Makes `lds` bytes of dynamic LDS launchable for `kernel` on the current
// device: up to 64 KiB needs nothing; above, the kernel's dynamic limit is
// raised, once per kernel and device, to the workgroup maximum (160 KiB on
// gfx950) minus the kernel's static LDS.  Returns the runtime's error, or
// hipErrorInvalidValue if the request cannot fit.
inline hipError_t allow_lds(const void *kernel, int64_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({kernel, dev})) return hipSuccess;
    hipFuncAttributes fa{};
    e = hipFuncGetAttributes(&fa, kernel);
    if (e != hipSuccess) return e;
    const int64_t room = int64_t(160 * 1024) - int64_t(fa.sharedSizeBytes);
    if (lds > room) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(room));
    if (e == hipSuccess) done.insert({kernel, dev});
    return e;
}

// One kernel launch of the LF2D loop: HIER covers launch positions
// [begin, end) of one block colour; GCOL covers slots [begin, end) of one
// colour; ATOMIC and DEBUG cover elements [0, end - begin).
hipError_t lf2d_launch_one(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                           int64_t lds_bytes);

// The same for the hex element loop (x in x, v in q, force in res, kappa in
// gm1; emap holds 8 node ids per slot).
hipError_t hex_launch_one(const LaunchArgs &la, int which, int32_t begin, int32_t end,
                          int64_t lds_bytes);

// One launch of a time-step loop (`kernel` a um_kernel value).  ADT:
// DIRECT over cells [0, end).  BOUNDARY_FLUX: GCOL over slots [begin, end)
// of one colour or ATOMIC over [0, end); emap holds (cell, a, b, 0) per
// slot.  UPDATE: DIRECT over cells [0, end) writing n_partials sums, then
// REDUCE adding their sum to gbl.  x, q and adt are double or float per
// dtype; res and gbl are double.
hipError_t step_launch_one(const LaunchArgs &la, int32_t kernel, int which, int32_t begin,
                           int32_t end);

// p[0..n) = 0 with a kernel on `stream`.
hipError_t zero_words(int32_t *p, int64_t n, hipStream_t stream);
// *dst += *src (device-scope atomic) with a one-lane kernel on `stream`.
hipError_t add_count(int32_t *dst, const int32_t *src, hipStream_t stream);

// dst[k] = src[idx[k]] for k < n over dim components (gather).
hipError_t permute_gather(const void *src, void *dst, const int32_t *idx, int64_t n, int32_t dim,
                          int32_t dtype, int32_t layout, hipStream_t stream);

}  // namespace um
