// Grid-wide barrier of a cooperative launch (all workgroups resident).
#pragma once

#include "internal.h"

namespace grid {

constexpr int SLOTS = 8;   // first-level arrival counters
constexpr int LINE = 64;   // int32 per 256-byte line

// Barrier state, zero before the launch.  Workgroup g arrives at slot
// g mod 8 (one counter per 256-byte line, so that the slots' atomics
// proceed in parallel); the last arrival of each slot arrives at the top
// counter, and the last of those advances every slot's generation flag,
// which the workgroups of that slot poll.
struct GridBar {
    int32_t count[SLOTS][LINE];
    int32_t top[LINE];
    int32_t gen[SLOTS][LINE];
    int32_t abort[LINE];
};
constexpr size_t BAR_BYTES = sizeof(GridBar);
constexpr size_t BAR_WORDS = BAR_BYTES / 4;

// All workgroups of a cooperative launch meet here.  Stores before the
// barrier are written back (release) and caches are refreshed after it
// (acquire), once per workgroup: every wave waits for its own stores, the
// workgroup meets, and one thread does the device-scope release, the
// arrival, the wait and the device-scope acquire for all of them.  A
// bounded spin turns a stuck barrier into an abort.
__device__ inline bool grid_sync(GridBar *b, int64_t limit) {
    __shared__ int32_t ok;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads and stores are complete
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int32_t G = (int32_t)gridDim.x, slots = G < SLOTS ? G : SLOTS;
        const int32_t x = (int32_t)blockIdx.x % slots, members = (G - x + slots - 1) / slots;
        int32_t good = 1;
        const int32_t g = __hip_atomic_load(&b->gen[x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool released = false;
        // (fence-to-fence synchronisation: each release fence above is
        // acquired by the fence of whoever reads its arrival, and passed on)
        if (__hip_atomic_fetch_add(&b->count[x][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == members) {
            // last of the slot: reset it and carry the slot's releases to the top counter
            __hip_atomic_store(&b->count[x][0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if (__hip_atomic_fetch_add(&b->top[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == slots) {
                __hip_atomic_store(&b->top[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                for (int32_t s = 0; s < slots; ++s)
                    __hip_atomic_store(&b->gen[s][0], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            int64_t spins = 0;
            while (__hip_atomic_load(&b->gen[x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&b->abort[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > limit) {
                    __hip_atomic_store(&b->abort[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    const bool res = ok != 0;
    __syncthreads();
    return res;
}

}  // namespace grid
