// (max, min) tile primitives shared by the closure kernels: element lane
// traits, the B x B tile product held in registers, and the register-resident
// closure of one diagonal tile.  Device code only; included by the kernels
// that run the blocked Floyd-Warshall recurrence.
#pragma once

#include "internal.h"

namespace fw {

typedef __attribute__((ext_vector_type(2))) unsigned short us2;

// Tile operands in device memory may be plain pointers or pointers qualified
// with the global address space (then every access is a global_* instruction
// rather than a flat one).  retype<U>(p) reinterprets p as a pointer to U in
// the same address space.
#define FW_GLOBAL __attribute__((address_space(1)))
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));  // 16 bytes, not a class type
template <typename U, typename T>
__device__ __forceinline__ U *retype(T *p) {
    return reinterpret_cast<U *>(p);
}
template <typename U, typename T>
__device__ __forceinline__ FW_GLOBAL U *retype(FW_GLOBAL T *p) {
    return (FW_GLOBAL U *)p;
}

template <typename E>
struct Lane;
template <>
struct Lane<int32_t> {
    using W = int32_t;  // one element per 32-bit lane
    static constexpr int PER = 1;
    __device__ static W splat(int32_t v) { return v; }
    __device__ static W relax(W c, W a, W b) { return max(c, min(a, b)); }
};
template <>
struct Lane<uint16_t> {
    using W = us2;  // two elements per 32-bit lane
    static constexpr int PER = 2;
    __device__ static W splat(uint16_t v) { return us2{v, v}; }
    __device__ static W relax(W c, W a, W b) {
        return __builtin_elementwise_max(c, __builtin_elementwise_min(a, b));
    }
};


// ------------------------------------------------------------------ tile product
// 256 threads as 16 x 16; thread (ty, tx) owns rows ty*TM .. and columns
// tx*TN .. of the C tile, held as TM x WN lanes.
template <typename E, int B>
struct Cfg {
    static constexpr int PER = Lane<E>::PER;
    static constexpr int TM = B / 16;
    static constexpr int TN = B / 16;
    static constexpr int WN = TN / PER;
    static constexpr int KC = sizeof(E) == 2 ? (B < 64 ? B : 64) : 32;  // k per LDS stage
    static constexpr int LA = KC + 16 / (int)sizeof(E);                 // padded pitches keep
    static constexpr int LB = B + 16 / (int)sizeof(E);                  // 16-byte row alignment
    static constexpr int LDS_ELEMS = B * LA + KC * LB;
};

template <typename E, int B>
struct Acc {
    typename Lane<E>::W c[Cfg<E, B>::TM][Cfg<E, B>::WN];
};

template <typename E, typename SrcP>
__device__ inline void copy_block(E *__restrict__ dst, int dst_pitch, SrcP src, int64_t src_pitch, int rows,
                                  int cols) {
    // cols * sizeof(E) is a multiple of 16; rows of src and dst are 16-byte aligned
    const int vpr = cols * (int)sizeof(E) / 16;
    for (int v = threadIdx.x; v < rows * vpr; v += 256) {
        const int rr = v / vpr, cv = v % vpr;
        const v4u32 x = *retype<const v4u32>(src + rr * src_pitch + cv * (16 / sizeof(E)));
        *reinterpret_cast<v4u32 *>(dst + rr * dst_pitch + cv * (16 / sizeof(E))) = x;
    }
}

template <typename E, int B, typename SrcP>
__device__ inline void acc_load(Acc<E, B> &a, SrcP src, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int ii = 0; ii < C::TM; ++ii) {
        const auto row = retype<const W>(src + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) a.c[ii][jj] = row[jj];
    }
}

template <typename E, int B, typename DstP>
__device__ inline void acc_store(const Acc<E, B> &a, DstP dst, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int ii = 0; ii < C::TM; ++ii) {
        const auto row = retype<W>(dst + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) row[jj] = a.c[ii][jj];
    }
}

// a = max(a, A (x) Bm) with A, Bm B x B tiles in global memory (row pitches
// lda, ldb).  lds holds Cfg::LDS_ELEMS elements.  Starts and ends with a
// barrier, so A or Bm may be the tile that the caller overwrites afterwards.
template <typename E, int B, typename PA, typename PB>
__device__ inline void acc_product(Acc<E, B> &a, PA A, int64_t lda, PB Bm, int64_t ldb, E *lds) {
    using C = Cfg<E, B>;
    using L = Lane<E>;
    using W = typename L::W;
    constexpr int TM = C::TM, TN = C::TN, WN = C::WN, KC = C::KC, LA = C::LA, LB = C::LB;
    E *As = lds;
    E *Bs = lds + B * LA;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int kc = 0; kc < B; kc += KC) {
        __syncthreads();
        copy_block<E>(As, LA, A + kc, lda, B, KC);
        copy_block<E>(Bs, LB, Bm + (int64_t)kc * ldb, ldb, KC, B);
        __syncthreads();
        if constexpr (sizeof(E) == 4) {
            // four k per step: A values come as one 16-byte read per row
#pragma unroll 1
            for (int k = 0; k < KC; k += 4) {
                int4 av[TM];
                for (int ii = 0; ii < TM; ++ii) av[ii] = *reinterpret_cast<const int4 *>(&As[(ty * TM + ii) * LA + k]);
#pragma unroll
                for (int kp = 0; kp < 4; kp += 2) {
                    E b0[TN], b1[TN];
                    for (int jj = 0; jj < TN; jj += 4) {
                        const int4 x0 = *reinterpret_cast<const int4 *>(&Bs[(k + kp) * LB + tx * TN + jj]);
                        const int4 x1 = *reinterpret_cast<const int4 *>(&Bs[(k + kp + 1) * LB + tx * TN + jj]);
                        b0[jj] = x0.x, b0[jj + 1] = x0.y, b0[jj + 2] = x0.z, b0[jj + 3] = x0.w;
                        b1[jj] = x1.x, b1[jj + 1] = x1.y, b1[jj + 2] = x1.z, b1[jj + 3] = x1.w;
                    }
                    for (int ii = 0; ii < TM; ++ii) {
                        const E a0 = kp == 0 ? av[ii].x : av[ii].z;
                        const E a1 = kp == 0 ? av[ii].y : av[ii].w;
                        for (int jj = 0; jj < TN; ++jj)
                            a.c[ii][jj] = max(a.c[ii][jj], max(min(a0, b0[jj]), min(a1, b1[jj])));
                    }
                }
            }
        } else {
            // four k per step: A values come as one 8-byte read per row
#pragma unroll 1
            for (int k = 0; k < KC; k += 4) {
                uint2 av[TM];
                for (int ii = 0; ii < TM; ++ii) av[ii] = *reinterpret_cast<const uint2 *>(&As[(ty * TM + ii) * LA + k]);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    W bp[WN];
                    for (int jj = 0; jj < WN; ++jj)
                        bp[jj] = *reinterpret_cast<const W *>(&Bs[(k + kk) * LB + tx * TN + 2 * jj]);
                    for (int ii = 0; ii < TM; ++ii) {
                        const uint32_t word = kk < 2 ? av[ii].x : av[ii].y;
                        const unsigned short av16 = (kk & 1) ? (unsigned short)(word >> 16) : (unsigned short)word;
                        const W aa = L::splat(av16);
                        for (int jj = 0; jj < WN; ++jj) a.c[ii][jj] = L::relax(a.c[ii][jj], aa, bp[jj]);
                    }
                }
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ diagonal tile
// Plain recurrence over the tile's own vertices, elements held in registers:
// thread (ty, tx) owns rows ty + 16a and columns tx + 16b (a, b < B/16).
// Before step k the owners of row k and column k put them into LDS (double
// buffered, in thread order so each thread reads its values contiguously);
// row and column k do not change in step k, so one barrier per step
// suffices.  Steps run as B/16 unrolled groups of 16 so that the register
// index of row/column k (= k / 16) is a compile-time constant.
template <typename E>
__device__ inline E lane_get(const typename Lane<E>::W *v, int b) {
    if constexpr (sizeof(E) == 4) {
        return v[b];
    } else {
        return (b & 1) ? v[b >> 1].y : v[b >> 1].x;
    }
}

template <typename E, int B>
struct Diag {
    using L = Lane<E>;
    using W = typename L::W;
    static constexpr int RA = B / 16;       // rows per thread
    static constexpr int CW = B / 16;       // columns per thread
    static constexpr int WC = CW / L::PER;  // lanes per row

    // row and column 16 * KB + kk go to LDS slot `slot`
    template <int KB>
    __device__ __attribute__((always_inline)) static void publish(const W (&v)[RA][WC], int kk, int slot, int tx,
                                                                  int ty, E *rowbuf, E *colbuf) {
        if (ty == kk) {
            W *rb = reinterpret_cast<W *>(rowbuf + slot * B + tx * CW);
            for (int c = 0; c < WC; ++c) rb[c] = v[KB][c];
        }
        if (tx == kk) {
            for (int a = 0; a < RA; ++a) colbuf[slot * B + ty * RA + a] = lane_get<E>(v[a], KB);
        }
    }

    // steps k = 16 * KB .. 16 * KB + 15, then the next group
    template <int KB>
    __device__ __attribute__((always_inline)) static void steps(W (&v)[RA][WC], int tx, int ty, E *rowbuf,
                                                                E *colbuf) {
#pragma unroll 1
        for (int kk = 0; kk < 16; ++kk) {
            const int slot = kk & 1;  // k = 16 KB + kk has the parity of kk
            __syncthreads();
            W rk[WC];
            const W *rb = reinterpret_cast<const W *>(rowbuf + slot * B + tx * CW);
            for (int c = 0; c < WC; ++c) rk[c] = rb[c];
            for (int a = 0; a < RA; ++a) {
                const W ck = L::splat(colbuf[slot * B + ty * RA + a]);
                for (int c = 0; c < WC; ++c) v[a][c] = L::relax(v[a][c], ck, rk[c]);
            }
            if (kk < 15) {
                publish<KB>(v, kk + 1, slot ^ 1, tx, ty, rowbuf, colbuf);
            } else {
                if constexpr (KB + 1 < B / 16) publish<KB + 1>(v, 0, slot ^ 1, tx, ty, rowbuf, colbuf);
            }
        }
        if constexpr (KB + 1 < B / 16) steps<KB + 1>(v, tx, ty, rowbuf, colbuf);
    }
};

template <typename E, int B, typename SrcP, typename DstP>
__device__ inline void diag_close(SrcP src, int64_t lds_, DstP dst, int64_t ldd_, E *__restrict__ dst2, int64_t ldd2,
                                  E *buf) {
    using D = Diag<E, B>;
    using W = typename D::W;
    E *rowbuf = buf;          // [2][B]: thread tx's columns at tx*CW ..
    E *colbuf = buf + 2 * B;  // [2][B]: thread ty's rows at ty*RA ..
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    // the tile may just have been stored by other threads of the workgroup
    // (with another thread-to-element map)
    __syncthreads();
    W v[D::RA][D::WC];
    for (int a = 0; a < D::RA; ++a) {
        const auto row = src + (int64_t)(ty + 16 * a) * lds_ + tx;
        for (int c = 0; c < D::WC; ++c) {
            if constexpr (sizeof(E) == 4) {
                v[a][c] = row[16 * c];
            } else {
                v[a][c] = us2{row[16 * (2 * c)], row[16 * (2 * c + 1)]};
            }
        }
    }
    D::template publish<0>(v, 0, 0, tx, ty, rowbuf, colbuf);
    D::template steps<0>(v, tx, ty, rowbuf, colbuf);
    for (int a = 0; a < D::RA; ++a) {
        const auto row = dst + (int64_t)(ty + 16 * a) * ldd_ + tx;
        E *row2 = dst2 ? dst2 + (int64_t)(ty + 16 * a) * ldd2 + tx : nullptr;
        for (int b = 0; b < D::CW; ++b) {
            const E x = lane_get<E>(v[a], b);
            row[16 * b] = x;
            if (row2) row2[16 * b] = x;
        }
    }
    __syncthreads();
}

}  // namespace fw
