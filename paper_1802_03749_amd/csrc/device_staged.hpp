// Device helpers shared by the hierarchical kernels.
//
// Staged point ids of a block inside the hierarchical kernels.  A block's
// sorted staged list is stored either explicitly or, when it splits into few
// runs of consecutive ids, as run descriptors (first id, first staged
// position).  Run descriptors are loaded with one vector load per wave (lane
// r holds run r) and looked up with readlane, so resolving an id needs no
// chain of dependent memory loads.  Included by the HIP kernel files only.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace um {
namespace dev {

struct StagedIds {
    int32_t start, local;  // this lane's run descriptor (lanes < nr)
    int32_t nr;            // number of runs, 0 = explicit list
    const int32_t *__restrict__ list;

    // Called by every lane of the wave.  The planner only uses runs when nr
    // does not exceed the lanes of the block's smallest wave.
    __device__ __forceinline__ void init(const Run *__restrict__ runs, int32_t r0, int32_t n,
                                         const int32_t *__restrict__ explicit_list) {
        nr = n;
        list = explicit_list;
        const int lane = int(threadIdx.x & 63u);
        start = 0;
        local = 0;
        if (lane < n) {
            const Run R = runs[r0 + lane];
            start = R.start;
            local = R.local;
        }
    }

    // Id at staged position t (runs are sorted by `local`; the first is 0).
    __device__ __forceinline__ int32_t operator()(int t) const {
        if (nr == 0) return list[t];
        int32_t g = 0;
        for (int r = 0; r < nr; ++r) {
            const int32_t l = __builtin_amdgcn_readlane(local, r);
            const int32_t s = __builtin_amdgcn_readlane(start, r);
            if (t >= l) g = s + (t - l);
        }
        return g;
    }
};

// Dataflow schedules: waits until the completion flag *fl holds `epoch`.
// Gives up after `ticks` of s_memrealtime (100 MHz), or at once when another
// wait of the same execution has given up (ctl[1] == epoch); a timeout adds
// one to ctl[0] and records its epoch in ctl[1].  Each execution has its own
// epoch, so a timeout never shortens the waits of a later execution.
__device__ __forceinline__ void bounded_wait(const int32_t *fl, int32_t epoch, int32_t *ctl,
                                             uint64_t ticks) {
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
        if (__builtin_amdgcn_s_memrealtime() - t_begin > ticks) {
            __hip_atomic_fetch_add(ctl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctl + 1, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

}  // namespace dev
}  // namespace um
