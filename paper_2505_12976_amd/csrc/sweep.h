// Frontier sweeps of a monotone (max, combine) relaxation over the rows of a
// dense m x m matrix A (row pitch ld), run to the fixpoint inside one
// cooperative launch:
//     x[j] <- max(x[j], max over i in F of comb(x[i], A[i][j])),
// where F holds the vertices whose value grew in the previous sweep.  Values
// only grow and each is the value of some path, so updating x in place (a
// row may see a value that grew earlier in the same sweep) reaches the same
// fixpoint: a vertex whose value grows is relaxed again in the next sweep,
// and a sweep that changes nothing ends the iteration with every row relaxed
// at its final value.  One launch can run NP independent problems of the
// same size side by side (the two directions of a widest-path check or of
// label propagation), sharing the barriers.
//
// Layout: the column blocks of all problems (1024 columns each: a lane
// reads 16 of them as 16-byte vectors, each vector load of a wavefront one
// contiguous kilobyte of the row) are spread over the workgroups, with a
// share of the frontier rows per workgroup; its four wavefronts take every
// fourth frontier row of that share, four rows in flight at a time.
// (Blocks of a kilobyte per row or more keep the reads near the streaming
// rate; 256-column blocks reached about half of it.)  Partial maxima go to
// x with atomicMax, and a column whose value grew is appended to the next
// frontier at once: stamp[j] holds the last sweep whose list took j, so
// each vertex enters a list once whatever the number of workgroups that
// raise it.  One grid barrier per sweep.
#pragma once

#include "grid.h"

namespace sweep {

constexpr int CPL = 16;            // columns per lane
constexpr int CB = 64 * CPL;       // columns per block
constexpr int U = 4;               // frontier rows in flight per wavefront

// Workgroups for NP problems of m candidates: one share of the frontier
// per 256 rows of each column block, at most `cap` (the resident limit of
// the cooperative launch); small matrices take few workgroups, so that
// their barriers stay cheap.  Every column block of every problem gets at
// least one workgroup as long as cap >= NP * ceil(m / 1024), which holds
// for m <= 65535 and cap >= 128.
inline int64_t grid_size(int32_t m, int np, int64_t cap) {
    const int64_t ncb = (m + CB - 1) / CB;
    const int64_t g = np * ncb * ((m + 255) / 256);
    return g < 1 ? 1 : (g < cap ? g : cap);
}

// Rows of a matrix at p with pitch ld can be read as 16-byte vectors.
template <typename E>
inline bool vec_ok(const void *p, int64_t ld) {
    return reinterpret_cast<uintptr_t>(p) % 16 == 0 && (ld * (int64_t)sizeof(E)) % 16 == 0;
}

// Elements per 16-byte vector and vectors per lane.
template <typename E>
constexpr int vlen() {
    return 16 / (int)sizeof(E);
}
template <typename E>
constexpr int nvec() {
    return CPL / vlen<E>();
}

// Column (relative to the block) of element c of a lane's share: vector
// k = c / V covers columns (64 k + lane) V .. + V.
template <typename E>
__device__ inline int32_t lane_col(int lane, int c) {
    constexpr int V = vlen<E>();
    return ((c / V) * 64 + lane) * V + c % V;
}

// The lane's 16 elements of a row (row points at the block's first column).
// FULL: the whole block is inside the matrix and vector-aligned (16-byte
// loads); otherwise one element at a time, 0 past `valid` columns.  The
// choice is made per block, never per lane: a per-lane choice made the
// compiler wait for every earlier load before each vector load.
template <typename E, bool FULL>
__device__ inline void load_row(const E *__restrict__ row, int32_t valid, int lane, uint32_t (&v)[CPL]) {
    constexpr int V = vlen<E>();
    for (int k = 0; k < nvec<E>(); ++k) {
        const int32_t c0 = (k * 64 + lane) * V;
        if constexpr (FULL) {
            const uint4 q = *reinterpret_cast<const uint4 *>(row + c0);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
            if constexpr (sizeof(E) == 4) {
                for (int u = 0; u < 4; ++u) v[k * V + u] = w[u];
            } else {
                for (int u = 0; u < 4; ++u) {
                    v[k * V + 2 * u] = w[u] & 0xFFFFu;
                    v[k * V + 2 * u + 1] = w[u] >> 16;
                }
            }
        } else {
            for (int u = 0; u < V; ++u) v[k * V + u] = c0 + u < valid ? (uint32_t)row[c0 + u] : 0u;
        }
    }
}

// One problem of a launch (device pointers).
template <typename X, typename E>
struct Problem {
    const E *A;          // rows, pitch ld
    int64_t ld;
    int32_t vec;         // A can be read as 16-byte vectors (vec_ok)
    X *x;                // m values, updated in place (set by the caller's init)
    int32_t *stamp;      // m: the last sweep (from 1) whose list took the vertex; 0 on entry
    int32_t *front[2];   // frontier lists of m entries; front[0] holds the first frontier
    int32_t *count;      // [0..2] list sizes by sweep mod 3 ([0] the first frontier's, [1], [2] zero
                         // on entry); [3] sweeps with a non-empty frontier (zero on entry)
};

template <typename X, typename E, int NP>
struct Run {
    Problem<X, E> p[NP];
    int32_t max_sweeps;  // more means a broken invariant (device error)
    grid::GridBar *bar;
    int32_t *err;
    int64_t spin_limit;
};

// Counter address of problem q's count slot c (q, c uniform).
template <typename X, typename E, int NP>
__device__ inline int32_t *count_at(const Run<X, E, NP> &r, int q, int c) {
    return (NP > 1 && q) ? r.p[NP - 1].count + c : r.p[0].count + c;
}

// The sweeps.  comb(q, xi, a) combines a row value with an entry a of
// problem q's matrix (returning 0 when nothing passes; q is uniform over a
// workgroup); accept(j) says whether column j may take values.  Returns false if a barrier gave up or the sweep bound was
// passed (the caller records the error).
template <typename X, typename E, int NP, typename Comb, typename Accept>
__device__ bool run(const Run<X, E, NP> &r, int32_t m, Comb comb, Accept accept) {
    static_assert(NP == 1 || NP == 2, "one or two problems per launch");
    __shared__ X part[4][CB];
    const int32_t G = gridDim.x, g = blockIdx.x;
    const int32_t ncb = (m + CB - 1) / CB, nblk = NP * ncb;
    const int32_t shares = G >= nblk ? G / nblk : 1;
    const bool active = g < nblk * shares;
    const int32_t blk = g % nblk, share = g / nblk;
    const int q = NP > 1 ? blk / ncb : 0;  // this workgroup's problem
    const int32_t cb = blk % ncb;
    // (select, not index: a dynamically indexed array of the struct would live in scratch memory)
    const E *const A = (NP > 1 && q) ? r.p[NP - 1].A : r.p[0].A;
    const int64_t ld = (NP > 1 && q) ? r.p[NP - 1].ld : r.p[0].ld;
    const int32_t vec = (NP > 1 && q) ? r.p[NP - 1].vec : r.p[0].vec;
    X *const x = (NP > 1 && q) ? r.p[NP - 1].x : r.p[0].x;
    int32_t *const stamp = (NP > 1 && q) ? r.p[NP - 1].stamp : r.p[0].stamp;
    int32_t *const f0 = (NP > 1 && q) ? r.p[NP - 1].front[0] : r.p[0].front[0];
    int32_t *const f1 = (NP > 1 && q) ? r.p[NP - 1].front[1] : r.p[0].front[1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t blk0 = cb * CB;
    const int32_t valid = m - blk0;  // columns of this block inside the matrix
    const bool full = vec != 0 && valid >= CB;
    for (int32_t t = 0;; ++t) {
        // list sizes of this sweep: final since the last barrier
        int32_t nf = 0, any = 0;
        for (int qq = 0; qq < NP; ++qq) {
            const int32_t c = __hip_atomic_load(count_at(r, qq, t % 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            any |= c;
            if (qq == q) nf = c;
        }
        if (any == 0) break;
        if (t >= r.max_sweeps) {  // values only grow, so this cannot happen
            if (threadIdx.x == 0) set_device_error(r.err, SCHULZE_EDEVICE);
            return false;
        }
        if (g == 0 && threadIdx.x == 0)
            for (int qq = 0; qq < NP; ++qq) {
                // the list two sweeps ahead (read in the previous sweep, appended to in the next)
                *count_at(r, qq, (t + 2) % 3) = 0;
                if (*count_at(r, qq, t % 3)) ++*count_at(r, qq, 3);
            }
        const int32_t *F = (t & 1) ? f1 : f0;
        int32_t *Fn = (t & 1) ? f0 : f1;
        int32_t *cnt_next = count_at(r, q, (t + 1) % 3);
        if (active) {
            X best[CPL] = {};
            const int32_t step = 4 * shares;
            // The frontier indices of the next batch are loaded while the
            // rows of the current one are in flight, so that each batch
            // waits for one round trip to memory, not two.
            int32_t idx[U];
            auto load_idx = [&](int32_t q0, int32_t(&id)[U]) {
                for (int u = 0; u < U; ++u) {
                    const int32_t qi = q0 + u * step;
                    id[u] = qi < nf ? F[qi] : -1;
                }
            };
            int32_t q0 = share * 4 + wave;
            load_idx(q0, idx);
            for (; q0 < nf; q0 += U * step) {
                // rows first, then their values and the next indices: all
                // in flight together, one wait before the arithmetic
                uint32_t a[U][CPL];
                if (full) {
                    for (int u = 0; u < U; ++u)
                        load_row<E, true>(A + (int64_t)(idx[u] < 0 ? 0 : idx[u]) * ld + blk0, valid, lane, a[u]);
                } else {
                    for (int u = 0; u < U; ++u)
                        load_row<E, false>(A + (int64_t)(idx[u] < 0 ? 0 : idx[u]) * ld + blk0, valid, lane, a[u]);
                }
                X xi[U];
                for (int u = 0; u < U; ++u) xi[u] = idx[u] < 0 ? (X)0 : x[idx[u] < 0 ? 0 : idx[u]];
                load_idx(q0 + U * step, idx);
                for (int u = 0; u < U; ++u)
                    for (int c = 0; c < CPL; ++c) best[c] = max(best[c], comb(q, xi[u], a[u][c]));
            }
            for (int c = 0; c < CPL; ++c) part[wave][lane_col<E>(lane, c)] = best[c];
        }
        __syncthreads();
        if (active) {
            for (int c = 0; c < CB / 256; ++c) {
                const int32_t jl = c * 256 + threadIdx.x, j = blk0 + jl;
                bool add = false;
                if (j < m && accept(j)) {
                    const X v = max(max(part[0][jl], part[1][jl]), max(part[2][jl], part[3][jl]));
                    if (v > x[j] && atomicMax(&x[j], v) < v) add = atomicMax(&stamp[j], t + 1) < t + 1;
                }
                const uint64_t bal = __ballot(add);
                int32_t base = 0;
                if (lane == 0 && bal) base = atomicAdd(cnt_next, (int32_t)__popcll(bal));
                base = __shfl(base, 0);
                if (add) Fn[base + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = j;
            }
        }
        if (!grid::grid_sync(r.bar, r.spin_limit)) return false;
    }
    return true;
}

}  // namespace sweep
