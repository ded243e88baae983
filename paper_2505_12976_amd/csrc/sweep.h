// Frontier sweeps of a monotone (max, combine) relaxation over the rows of a
// dense m x m matrix A (row pitch ld), run to the fixpoint inside one
// cooperative launch:
//     x[j] <- max(x[j], max over i in F of comb(x[i], A[i][j])),
// where F holds the vertices whose value grew in the previous sweep.  Values
// only grow and each is the value of some path, so updating x in place (a
// row may see a value that grew earlier in the same sweep) reaches the same
// fixpoint: a vertex whose value grows is relaxed again in the next sweep,
// and a sweep that changes nothing ends the iteration with every row relaxed
// at its final value.
//
// Layout: workgroup g takes column block g mod NCB (256 columns, four per
// lane, read as one 8- or 16-byte access) and row share g / NCB of the
// frontier; its four wavefronts take every fourth frontier row of that
// share, eight rows in flight at a time.  Partial maxima go to x with
// atomicMax (at most one per column, share and sweep), a column whose value
// grew is flagged, and after a grid barrier the first share's workgroup of
// each column block turns its flags into the next frontier.
#pragma once

#include "grid.h"

namespace sweep {

constexpr int CPL = 4;             // columns per lane
constexpr int CB = 64 * CPL;       // columns per block
constexpr int UNROLL = 8;          // frontier rows in flight per wavefront

// Workgroups for m candidates: one share of the frontier per 256 rows of
// each column block, at most `cap` (the resident limit of the cooperative
// launch); small matrices take few workgroups, so that their many barriers
// stay cheap.
inline int64_t grid_size(int32_t m, int64_t cap) {
    const int64_t ncb = (m + CB - 1) / CB;
    const int64_t g = ncb * ((m + 255) / 256);
    return g < 1 ? 1 : (g < cap ? g : cap);
}

// Four consecutive elements of a row starting at a multiple of 4.
template <typename E>
__device__ inline void load4(const E *__restrict__ p, bool vec, int32_t valid, uint32_t (&v)[CPL]) {
    if (vec && valid >= CPL) {
        if constexpr (sizeof(E) == 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(p);
            v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
        } else {
            const uint2 q = *reinterpret_cast<const uint2 *>(p);
            v[0] = q.x & 0xFFFFu, v[1] = q.x >> 16, v[2] = q.y & 0xFFFFu, v[3] = q.y >> 16;
        }
    } else {
        for (int c = 0; c < CPL; ++c) v[c] = c < valid ? (uint32_t)p[c] : 0u;
    }
}

// Shared state of one run (device pointers; fcount, changed zero on entry
// except as the caller's init sets them).
template <typename X>
struct Buffers {
    X *x;                // m values, updated in place
    int32_t *front[2];   // frontier lists
    int32_t *fcount;     // [0], [1] frontier sizes, [2] sweeps run
    uint8_t *changed;    // m flags
    grid::GridBar *bar;
    int32_t *err;
    int64_t spin_limit;
    int32_t max_sweeps;
};

// The sweeps.  comb(xi, a) combines a row value with an edge entry a
// (returning 0 when nothing passes); accept(j) says whether column j may
// take values.  Returns false if a barrier gave up (the caller records the
// error).
template <typename X, typename E, typename Comb, typename Accept>
__device__ bool run(const E *__restrict__ A, int64_t ld, int32_t m, bool vec, Buffers<X> &b, Comb comb,
                    Accept accept) {
    __shared__ X part[4][CB];
    const int32_t G = gridDim.x, g = blockIdx.x;
    const int32_t ncb = (m + CB - 1) / CB;
    const int32_t shares = G >= ncb ? G / ncb : 1;
    const bool active = g < ncb * shares;
    const int32_t cb = g % ncb, share = g / ncb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t col0 = cb * CB + lane * CPL;
    const int32_t valid = m - col0;  // columns of this lane inside the matrix (may be <= 0)
    int cur = 0;
    int32_t sweeps = 0;
    for (;;) {
        const int32_t nf = __hip_atomic_load(&b.fcount[cur], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (nf == 0) break;
        if (++sweeps > b.max_sweeps) {  // values only grow, so this cannot happen
            if (threadIdx.x == 0) set_device_error(b.err, SCHULZE_EDEVICE);
            break;
        }
        // (select, not index: a dynamically indexed array of the struct would live in scratch memory)
        const int32_t *F = cur ? b.front[1] : b.front[0];
        int32_t *Fn = cur ? b.front[0] : b.front[1];
        if (active) {
            X best[CPL] = {};
            const int32_t step = 4 * shares;
            for (int32_t q0 = share * 4 + wave; q0 < nf; q0 += UNROLL * step) {
                int32_t idx[UNROLL];
                for (int u = 0; u < UNROLL; ++u) {
                    const int32_t q = q0 + u * step;
                    idx[u] = q < nf ? F[q] : -1;
                }
                X xi[UNROLL];
                uint32_t a[UNROLL][CPL];
                for (int u = 0; u < UNROLL; ++u) {
                    const int32_t i = idx[u] < 0 ? 0 : idx[u];
                    xi[u] = idx[u] < 0 ? (X)0 : b.x[i];
                    load4<E>(A + (int64_t)i * ld + col0, vec, valid, a[u]);
                }
                for (int u = 0; u < UNROLL; ++u)
                    for (int c = 0; c < CPL; ++c) best[c] = max(best[c], comb(xi[u], a[u][c]));
            }
            for (int c = 0; c < CPL; ++c) part[wave][lane * CPL + c] = best[c];
        }
        __syncthreads();
        if (active) {
            const int32_t j = cb * CB + threadIdx.x;
            if (j < m && accept(j)) {
                const X v = max(max(part[0][threadIdx.x], part[1][threadIdx.x]),
                                max(part[2][threadIdx.x], part[3][threadIdx.x]));
                if (v > b.x[j] && atomicMax(&b.x[j], v) < v) b.changed[j] = 1;
            }
        }
        if (!grid::grid_sync(b.bar, b.spin_limit)) return false;
        // the next frontier: the columns that grew, collected by share 0
        if (active && share == 0) {
            const int32_t j = cb * CB + threadIdx.x;
            const bool grew = j < m && b.changed[j];
            if (grew) b.changed[j] = 0;
            const uint64_t bal = __ballot(grew);
            int32_t base = 0;
            if (lane == 0 && bal) base = atomicAdd(&b.fcount[cur ^ 1], (int32_t)__popcll(bal));
            base = __shfl(base, 0);
            if (grew) Fn[base + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = j;
        }
        if (g == 0 && threadIdx.x == 0) b.fcount[cur] = 0;  // the consumed list is the next target
        if (!grid::grid_sync(b.bar, b.spin_limit)) return false;
        cur ^= 1;
    }
    if (g == 0 && threadIdx.x == 0) b.fcount[2] = sweeps;
    return true;
}

}  // namespace sweep
