// 64 x 64 tiles between device memory and LDS, for the passes that need a
// block of a matrix next to its transposed block (edge weights, beats,
// per-candidate statistics).  Interior tiles of suitably aligned matrices
// move as 16-byte vectors (four or eight elements per access, so that many
// bytes are in flight per wavefront); edge tiles and unaligned matrices fall
// back to one element per access with bounds checks.  256 threads.
#pragma once

#include "internal.h"

namespace tio {

constexpr int T = 64;       // tile side
constexpr int PITCH = 65;   // LDS row pitch (odd: column reads hit distinct banks)

// 16-byte vector accesses are valid for a matrix at p with row pitch ld.
template <typename E>
inline bool vec_ok(const void *p, int64_t ld) {
    return p && (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((ld * (int64_t)sizeof(E)) % 16 == 0);
}

// The V elements of a 16-byte vector.
template <typename E>
__device__ inline void unpack(const uint4 &x, E *e);
template <>
__device__ inline void unpack<int32_t>(const uint4 &x, int32_t *e) {
    e[0] = (int32_t)x.x, e[1] = (int32_t)x.y, e[2] = (int32_t)x.z, e[3] = (int32_t)x.w;
}
template <>
__device__ inline void unpack<uint16_t>(const uint4 &x, uint16_t *e) {
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
    for (int u = 0; u < 4; ++u) {
        e[2 * u] = (uint16_t)(w[u] & 0xFFFFu);
        e[2 * u + 1] = (uint16_t)(w[u] >> 16);
    }
}
template <typename E>
__device__ inline uint4 pack(const E *e);
template <>
__device__ inline uint4 pack<int32_t>(const int32_t *e) {
    return make_uint4((uint32_t)e[0], (uint32_t)e[1], (uint32_t)e[2], (uint32_t)e[3]);
}
template <>
__device__ inline uint4 pack<uint16_t>(const uint16_t *e) {
    uint32_t w[4];
    for (int u = 0; u < 4; ++u) w[u] = (uint32_t)e[2 * u] | ((uint32_t)e[2 * u + 1] << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// t[r][c] = src[(r0 + r) ld + c0 + c], 0 where r0 + r >= rows or c0 + c >= cols.
template <typename E>
__device__ inline void load(E (*t)[PITCH], const E *__restrict__ src, int64_t ld, int32_t r0, int32_t c0,
                            int32_t rows, int32_t cols, bool vec) {
    if (vec && r0 + T <= rows && c0 + T <= cols) {
        constexpr int V = 16 / (int)sizeof(E);  // elements per vector
        constexpr int VPR = T / V;              // vectors per row
        constexpr int PER = T * VPR / 256;      // vectors per thread
        uint4 x[PER];
        for (int k = 0; k < PER; ++k) {  // all loads first, so that they are in flight together
            const int q = threadIdx.x + 256 * k;
            const int r = q / VPR, cv = q % VPR;
            x[k] = *reinterpret_cast<const uint4 *>(src + (int64_t)(r0 + r) * ld + c0 + cv * V);
        }
        for (int k = 0; k < PER; ++k) {
            const int q = threadIdx.x + 256 * k;
            const int r = q / VPR, cv = q % VPR;
            E e[V];
            unpack<E>(x[k], e);
            for (int u = 0; u < V; ++u) t[r][cv * V + u] = e[u];
        }
    } else {
        for (int q = threadIdx.x; q < T * T; q += 256) {
            const int r = q / T, c = q % T;
            t[r][c] = (r0 + r < rows && c0 + c < cols) ? src[(int64_t)(r0 + r) * ld + c0 + c] : (E)0;
        }
    }
}

// The same tile in two halves, so that the loads can be issued early and
// the LDS written later: fetch() loads the tile into registers, put()
// writes them to LDS.  VEC (the matrix is vector-aligned and its side a
// multiple of the vector length): 16-byte loads, rows and vectors past the
// edge read the tile's first row / vector instead, so that every tile takes
// the same loads (what lands outside the matrix is garbage, to be ignored
// by the caller).  Otherwise one element at a time, 0 outside.
template <typename E>
struct Regs {
    static constexpr int PER = T * (T / (16 / (int)sizeof(E))) / 256;  // 16-byte vectors per thread
    uint4 x[PER];
};

template <typename E, bool VEC>
__device__ inline void fetch(Regs<E> &g, const E *__restrict__ src, int64_t ld, int32_t r0, int32_t c0, int32_t rows,
                             int32_t cols) {
    constexpr int V = 16 / (int)sizeof(E), VPR = T / V;
    for (int k = 0; k < Regs<E>::PER; ++k) {
        const int q = threadIdx.x + 256 * k;
        int32_t r = r0 + q / VPR, c = c0 + (q % VPR) * V;
        if (VEC) {
            r = r < rows ? r : r0;
            c = c < cols ? c : c0;
            g.x[k] = *reinterpret_cast<const uint4 *>(src + (int64_t)r * ld + c);
        } else {
            E e[V];
            for (int u = 0; u < V; ++u) e[u] = (r < rows && c + u < cols) ? src[(int64_t)r * ld + c + u] : (E)0;
            g.x[k] = pack<E>(e);
        }
    }
}

template <typename E>
__device__ inline void put(E (*t)[PITCH], const Regs<E> &g) {
    constexpr int V = 16 / (int)sizeof(E), VPR = T / V;
    for (int k = 0; k < Regs<E>::PER; ++k) {
        const int q = threadIdx.x + 256 * k;
        E e[V];
        unpack<E>(g.x[k], e);
        for (int u = 0; u < V; ++u) t[q / VPR][(q % VPR) * V + u] = e[u];
    }
}

// dst[(r0 + r) ld + c0 + c] = f(r, c) for r0 + r < rows and c0 + c < cols.
template <typename E, typename F>
__device__ inline void store(E *__restrict__ dst, int64_t ld, int32_t r0, int32_t c0, int32_t rows, int32_t cols,
                             bool vec, F f) {
    if (vec && r0 + T <= rows && c0 + T <= cols) {
        constexpr int V = 16 / (int)sizeof(E);
        constexpr int VPR = T / V;
        for (int q = threadIdx.x; q < T * VPR; q += 256) {
            const int r = q / VPR, cv = q % VPR;
            E e[V];
            for (int u = 0; u < V; ++u) e[u] = f(r, cv * V + u);
            *reinterpret_cast<uint4 *>(dst + (int64_t)(r0 + r) * ld + c0 + cv * V) = pack<E>(e);
        }
    } else {
        for (int q = threadIdx.x; q < T * T; q += 256) {
            const int r = q / T, c = q % T;
            if (r0 + r < rows && c0 + c < cols) dst[(int64_t)(r0 + r) * ld + c0 + c] = f(r, c);
        }
    }
}

}  // namespace tio
