// Grid-wide barrier of a cooperative launch (all workgroups resident).
#pragma once

#include "internal.h"

namespace grid {

struct GridBar {  // zero on entry
    int32_t count;
    int32_t gen;
    int32_t abort;
};

// All workgroups of a cooperative launch meet here.  Stores before the
// barrier are written back (release) and caches are refreshed after it
// (acquire).  A bounded spin turns a stuck barrier into an abort.
__device__ inline bool grid_sync(GridBar *b, int64_t limit) {
    __shared__ int32_t ok;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t good = 1;
        const int32_t g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t arrived = __hip_atomic_fetch_add(&b->count, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (arrived == (int32_t)gridDim.x) {
            __hip_atomic_store(&b->count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&b->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int64_t spins = 0;
            while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > limit) {
                    __hip_atomic_store(&b->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        ok = good;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool res = ok != 0;
    __syncthreads();
    return res;
}

}  // namespace grid
