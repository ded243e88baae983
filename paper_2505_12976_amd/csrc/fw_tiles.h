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
#define FW_LDS __attribute__((address_space(3)))
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));  // 16 bytes, not a class type
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));  // 8 bytes
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

// p through a scalar register: the per-lane addresses built from it are
// rebuilt at each use instead of being kept live in vector registers
// across the products in between.
template <typename P>
__device__ __forceinline__ P scalar_ptr(P p) {
    const uint64_t u = (uint64_t)p;  // uniform: the same tile for every lane
    // (readfirstlane returns int: widen through uint32_t, never sign-extend)
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    asm volatile("" : "+s"(v));
    return (P)v;
}

// The thread index, opaque to the optimiser: per-lane offsets built from it
// are computed where they are used, not hoisted to the kernel's entry and
// kept live in vector registers for its whole run.
__device__ __forceinline__ int lane_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

template <typename E, int B, typename SrcP>
__device__ inline void acc_load(Acc<E, B> &a, SrcP src, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int t = lane_tid(), tx = t & 15, ty = t >> 4;
    src = scalar_ptr(src);
    for (int ii = 0; ii < C::TM; ++ii) {
        const auto row = retype<const W>(src + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) a.c[ii][jj] = row[jj];
    }
}

template <typename E, int B, typename DstP>
__device__ inline void acc_store(const Acc<E, B> &a, DstP dst, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int t = lane_tid(), tx = t & 15, ty = t >> 4;
    dst = scalar_ptr(dst);
    for (int ii = 0; ii < C::TM; ++ii) {
        const auto row = retype<W>(dst + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) row[jj] = a.c[ii][jj];
    }
}

// The four k of one step of the 16-bit product: A values av (four k per
// row, one 8-byte read each), B rows at bs (pitch ldb elements, this
// thread's columns).  The B row of step k+1 is read before the products of
// step k (the scheduling barrier keeps it there), so that only the first
// read of each step waits.
template <int B>
__device__ __forceinline__ void step4_16(Acc<uint16_t, B> &a, const v2u32 (&av)[Cfg<uint16_t, B>::TM],
                                         const FW_LDS uint16_t *bs, int ldb) {
    using C = Cfg<uint16_t, B>;
    using L = Lane<uint16_t>;
    using W = typename L::W;
    constexpr int TM = C::TM, WN = C::WN;
    W bq[2][WN];
    const FW_LDS W *b0 = (const FW_LDS W *)bs;
    for (int jj = 0; jj < WN; ++jj) bq[0][jj] = b0[jj];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        if (kk + 1 < 4) {
            const FW_LDS W *bn = (const FW_LDS W *)(bs + (kk + 1) * ldb);
            for (int jj = 0; jj < WN; ++jj) bq[(kk + 1) & 1][jj] = bn[jj];
        }
        __builtin_amdgcn_sched_barrier(0);
        const W *bp = bq[kk & 1];
        for (int ii = 0; ii < TM; ++ii) {
            const uint32_t word = kk < 2 ? av[ii].x : av[ii].y;
            const unsigned short av16 = (kk & 1) ? (unsigned short)(word >> 16) : (unsigned short)word;
            const W aa = L::splat(av16);
            // all mins of the row before its maxes: a max right after the
            // min it reads needs a wait state when that min takes the high
            // half of its operand (the compiler inserts an s_nop there)
            W t[WN];
            for (int jj = 0; jj < WN; ++jj) t[jj] = __builtin_elementwise_min(aa, bp[jj]);
            for (int jj = 0; jj < WN; ++jj) a.c[ii][jj] = __builtin_elementwise_max(a.c[ii][jj], t[jj]);
        }
    }
}

// Direct-to-LDS staging of the 16-bit product with B = 128: chunks of 32 k
// (an A chunk of B rows x 64 bytes and a B chunk of 32 rows x 256 bytes),
// double buffered, so that the next chunk streams into LDS while the
// current one is multiplied and no registers hold staged data.  Each
// wavefront instruction moves one contiguous kilobyte (lane l to byte 16 l),
// so the LDS rows are unpadded: the A reads of a wavefront hit four
// addresses (broadcast) and the B reads sixteen consecutive 16-byte groups.
struct Dma128 {
    static constexpr int B = 128, KC = 32;
    static constexpr int AS = B * KC, BS = KC * B;     // elements per chunk
    static constexpr int LDS_ELEMS = 2 * (AS + BS);    // two buffers
};

template <typename PA, typename PB>
__device__ __forceinline__ void dma_chunk128(PA A, int64_t lda, PB Bm, int64_t ldb, int kc, FW_LDS uint16_t *As,
                                             FW_LDS uint16_t *Bs) {
    const int t = lane_tid(), w = t >> 6, l = t & 63;
    // A: instruction i = rows 16 i .. 16 i + 15, four 16-byte pieces each
    for (int i = w; i < 8; i += 4)
        __builtin_amdgcn_global_load_lds(A + (int64_t)(16 * i + (l >> 2)) * lda + kc + (l & 3) * 8, As + i * 512, 16,
                                         0, 0);
    // B: instruction i = k rows 4 i .. 4 i + 3, sixteen 16-byte pieces each
    for (int i = w; i < 8; i += 4)
        __builtin_amdgcn_global_load_lds(Bm + (int64_t)(kc + 4 * i + (l >> 4)) * ldb + (l & 15) * 8, Bs + i * 512, 16,
                                         0, 0);
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
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    if constexpr (sizeof(E) == 2 && B == 128) {
        using D = Dma128;
        static_assert(D::LDS_ELEMS <= C::LDS_ELEMS, "LDS of the staged product");
        FW_LDS uint16_t *buf = (FW_LDS uint16_t *)lds;
        // (scalar operand addresses: the per-lane load addresses are built
        // here, not hoisted out of the caller's loops)
        A = scalar_ptr(A);
        Bm = scalar_ptr(Bm);
        __syncthreads();  // the previous user of the LDS is done
        dma_chunk128(A, lda, Bm, ldb, 0, buf, buf + D::AS);
#pragma unroll 1
        for (int c = 0; c < B / D::KC; ++c) {
            FW_LDS uint16_t *As = buf + (c & 1) * (D::AS + D::BS);
            FW_LDS uint16_t *Bs = As + D::AS;
            __builtin_amdgcn_s_waitcnt(0);  // this wave's pieces of chunk c are in LDS
            __syncthreads();                // everyone's are, and chunk c-1 is consumed
            if (c + 1 < B / D::KC) {
                FW_LDS uint16_t *An = buf + ((c + 1) & 1) * (D::AS + D::BS);
                dma_chunk128(A, lda, Bm, ldb, (c + 1) * D::KC, An, An + D::AS);
            }
#pragma unroll 1
            for (int k = 0; k < D::KC; k += 4) {
                v2u32 av[TM];
                for (int ii = 0; ii < TM; ++ii) av[ii] = *(const FW_LDS v2u32 *)(As + (ty * TM + ii) * D::KC + k);
                step4_16<B>(a, av, &Bs[k * B + tx * TN], B);
            }
        }
        __syncthreads();
        return;
    }
    E *As = lds;
    E *Bs = lds + B * LA;
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
                // c = max3(max3(c, m0, m1), m2, m3) with mi = min(a_i, b_i): the
                // four k of a step as two v_max3_i32 and four v_min_i32
                E bk[4][TN];
                for (int kp = 0; kp < 4; ++kp)
                    for (int jj = 0; jj < TN; jj += 4) {
                        const int4 x = *reinterpret_cast<const int4 *>(&Bs[(k + kp) * LB + tx * TN + jj]);
                        bk[kp][jj] = x.x, bk[kp][jj + 1] = x.y, bk[kp][jj + 2] = x.z, bk[kp][jj + 3] = x.w;
                    }
                for (int ii = 0; ii < TM; ++ii) {
                    const E a0 = av[ii].x, a1 = av[ii].y, a2 = av[ii].z, a3 = av[ii].w;
                    for (int jj = 0; jj < TN; ++jj) {
                        const E m0 = min(a0, bk[0][jj]), m1 = min(a1, bk[1][jj]);
                        const E m2 = min(a2, bk[2][jj]), m3 = min(a3, bk[3][jj]);
                        const E c1 = max(max(a.c[ii][jj], m0), m1);
                        a.c[ii][jj] = max(max(c1, m2), m3);
                    }
                }
            }
        } else {
            // four k per step: A values come as one 8-byte read per row; the
            // B row of step k+1 is read before the products of step k (the
            // scheduling barrier keeps it there), so that only the first read
            // of each step waits
#pragma unroll 1
            for (int k = 0; k < KC; k += 4) {
                uint2 av[TM];
                for (int ii = 0; ii < TM; ++ii) av[ii] = *reinterpret_cast<const uint2 *>(&As[(ty * TM + ii) * LA + k]);
                W bq[2][WN];
                for (int jj = 0; jj < WN; ++jj) bq[0][jj] = *reinterpret_cast<const W *>(&Bs[k * LB + tx * TN + 2 * jj]);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    if (kk + 1 < 4) {
                        for (int jj = 0; jj < WN; ++jj)
                            bq[(kk + 1) & 1][jj] = *reinterpret_cast<const W *>(&Bs[(k + kk + 1) * LB + tx * TN + 2 * jj]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    const W *bp = bq[kk & 1];
                    for (int ii = 0; ii < TM; ++ii) {
                        const uint32_t word = kk < 2 ? av[ii].x : av[ii].y;
                        const unsigned short av16 = (kk & 1) ? (unsigned short)(word >> 16) : (unsigned short)word;
                        const W aa = L::splat(av16);
                        // all mins of the row before its maxes: a max right after the
                        // min it reads needs a wait state when that min takes the high
                        // half of its operand (the compiler inserts an s_nop there)
                        W t[WN];
                        for (int jj = 0; jj < WN; ++jj) t[jj] = __builtin_elementwise_min(aa, bp[jj]);
                        for (int jj = 0; jj < WN; ++jj) a.c[ii][jj] = __builtin_elementwise_max(a.c[ii][jj], t[jj]);
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
// The steps run in blocks of S (4, or 2 for the larger tiles) with one
// barrier per block: before block k0 .. k0+S-1 the owners put rows and
// columns k0 .. k0+S-1 and the S x S block where they cross into LDS (double
// buffered), and every thread then runs the S steps on its own elements,
// carrying its private copies of those rows (at its columns), columns (at
// its rows) and the block through the same steps, so that step k0+s sees
// row and column k0+s as the earlier steps of the block left them.  The
// result is that of the plain recurrence, step by step.  Blocks run in B/16
// groups of 16 steps so that the register index of rows and columns k
// (= k / 16) is a compile-time constant.
template <typename E>
__device__ inline E lane_get(const typename Lane<E>::W *v, int b) {
    if constexpr (sizeof(E) == 4) {
        return v[b];
    } else {
        return (b & 1) ? v[b >> 1].y : v[b >> 1].x;
    }
}

// Steps per barrier of the diagonal closure: 4 where the tile's registers
// leave room for the copies, else 2; 1 for 16-bit tiles of 128, so that
// the closure call fits the register budget of four workgroups per CU.
template <typename E, int B>
constexpr int diag_steps() {
    return B <= 64 ? 4 : (sizeof(E) == 2 ? 1 : 2);
}

template <typename E, int B, int S_ = diag_steps<E, B>()>
struct Diag {
    using L = Lane<E>;
    using W = typename L::W;
    static constexpr int PER = L::PER;
    static constexpr int RA = B / 16;       // rows per thread
    static constexpr int CW = B / 16;       // columns per thread
    static constexpr int WC = CW / PER;     // lanes per row slice
    static constexpr int RP = RA / PER;     // lanes per column slice
    static constexpr int S = S_;            // steps per barrier
    // one LDS slot: S rows (thread tx's columns at tx*CW ..), S columns
    // (thread ty's rows at ty*RA ..), the S x S block; padded to 16 bytes,
    // so that the second slot keeps the rows' and columns' 4-byte (and
    // wider) accesses aligned whatever S is
    static constexpr int SLOT = (2 * S * B + S * S + 7) / 8 * 8;
    static constexpr int LDS_ELEMS = 2 * SLOT;
    static_assert(SLOT * sizeof(E) % 16 == 0 && B * sizeof(E) % 16 == 0, "aligned LDS slots and rows");

    // rows and columns 16 KB + kk .. + S-1 into the slot at q
    template <int KB>
    __device__ __attribute__((always_inline)) static void publish(const W (&v)[RA][WC], int kk, FW_LDS E *q, int tx,
                                                                  int ty) {
        const int sr = ty - kk, sc = tx - kk;
        const bool row_owner = sr >= 0 && sr < S, col_owner = sc >= 0 && sc < S;
        if (row_owner) {
            FW_LDS W *rb = (FW_LDS W *)(q + sr * B + tx * CW);
#pragma unroll
            for (int c = 0; c < WC; ++c) rb[c] = v[KB][c];
        }
        if (col_owner) {
            FW_LDS W *cb = (FW_LDS W *)(q + S * B + sc * B + ty * RA);
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                if constexpr (sizeof(E) == 4) {
                    cb[p] = v[p][KB];
                } else {
                    cb[p] = W{lane_get<E>(v[2 * p], KB), lane_get<E>(v[2 * p + 1], KB)};
                }
            }
            if (row_owner) q[2 * S * B + sr * S + sc] = lane_get<E>(v[KB], KB);
        }
    }

    // the S steps of one block, from the slot at q
    __device__ __attribute__((always_inline)) static void block(W (&v)[RA][WC], const FW_LDS E *q, int tx, int ty) {
        W cv[S][RP];  // columns k0 + s at this thread's rows
        W rv[S][WC];  // rows k0 + s at this thread's columns
        E d[S][S];    // the block
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const FW_LDS W *cb = (const FW_LDS W *)(q + S * B + s * B + ty * RA);
#pragma unroll
            for (int p = 0; p < RP; ++p) cv[s][p] = cb[p];
            const FW_LDS W *rb = (const FW_LDS W *)(q + s * B + tx * CW);
#pragma unroll
            for (int c = 0; c < WC; ++c) rv[s][c] = rb[c];
        }
        if constexpr (S > 1) {
            constexpr int NW = S * S * (int)sizeof(E) / 4;  // 4-byte words of the block (8-byte aligned)
            uint32_t wv[NW];
            const FW_LDS uint32_t *db = (const FW_LDS uint32_t *)(q + 2 * S * B);
#pragma unroll
            for (int u = 0; u < NW; ++u) wv[u] = db[u];
#pragma unroll
            for (int i = 0; i < S * S; ++i) {
                if constexpr (sizeof(E) == 4) {
                    d[i / S][i % S] = (E)wv[i];
                } else {
                    d[i / S][i % S] = (E)((i & 1) ? (wv[i >> 1] >> 16) : (wv[i >> 1] & 0xFFFFu));
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const W ck = L::splat(lane_get<E>(cv[s], a));
#pragma unroll
                for (int c = 0; c < WC; ++c) v[a][c] = L::relax(v[a][c], ck, rv[s][c]);
            }
#pragma unroll
            for (int s2 = s + 1; s2 < S; ++s2) {
                const W x = L::splat(d[s][s2]);
#pragma unroll
                for (int p = 0; p < RP; ++p) cv[s2][p] = L::relax(cv[s2][p], x, cv[s][p]);
                const W y = L::splat(d[s2][s]);
#pragma unroll
                for (int c = 0; c < WC; ++c) rv[s2][c] = L::relax(rv[s2][c], y, rv[s][c]);
            }
#pragma unroll
            for (int s2 = s + 1; s2 < S; ++s2)
#pragma unroll
                for (int s3 = s + 1; s3 < S; ++s3)
                    if (s2 != s3)
                        d[s2][s3] = (E)max((int32_t)d[s2][s3], min((int32_t)d[s2][s], (int32_t)d[s][s3]));
            __builtin_amdgcn_sched_barrier(0);  // one step at a time: bounded register demand
        }
    }

    // blocks k0 = 16 KB, 16 KB + 4, .., then the next group
    template <int KB>
    __device__ __attribute__((always_inline)) static void steps(W (&v)[RA][WC], int tx, int ty, FW_LDS E *buf) {
#pragma unroll 1
        for (int g = 0; g < 16 / S; ++g) {
            const int slot = g & 1;  // block (16 / S) KB + g has the parity of g
            __syncthreads();
            block(v, buf + slot * SLOT, tx, ty);
            if (g + 1 < 16 / S) {
                publish<KB>(v, S * (g + 1), buf + (slot ^ 1) * SLOT, tx, ty);
            } else {
                if constexpr (KB + 1 < B / 16) publish<KB + 1>(v, 0, buf + (slot ^ 1) * SLOT, tx, ty);
            }
        }
        if constexpr (KB + 1 < B / 16) steps<KB + 1>(v, tx, ty, buf);
    }
};

template <typename E, int B, int S, bool STAGE, typename SrcP, typename DstP>
__device__ __attribute__((always_inline)) inline void diag_close_body(SrcP src, int64_t lds_, DstP dst, int64_t ldd_,
                                                                 E *__restrict__ dst2, int64_t ldd2, E *buf) {
    using D = Diag<E, B, S>;
    using W = typename D::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    FW_LDS E *lb = (FW_LDS E *)buf;  // (an LDS address: local accesses, also in an outlined call)
    src = scalar_ptr(src);
    // the tile may just have been stored by other threads of the workgroup
    // (with another thread-to-element map)
    __syncthreads();
    W v[D::RA][D::WC];
    if constexpr (STAGE) {
        // through LDS: 16-byte loads of the tile, then each thread takes its
        // strided elements (few registers in flight)
        {
            constexpr int V = 16 / (int)sizeof(E);
            constexpr int VPR = B / V;
#pragma unroll 4
            for (int q = threadIdx.x; q < B * VPR; q += 256) {
                const int r = q / VPR, cv = q % VPR;
                *(FW_LDS v4u32 *)(lb + r * B + cv * V) = *retype<const v4u32>(src + (int64_t)r * lds_ + cv * V);
            }
        }
        __syncthreads();
        for (int a = 0; a < D::RA; ++a) {
            const FW_LDS E *row = lb + (ty + 16 * a) * B + tx;
            for (int c = 0; c < D::WC; ++c) {
                if constexpr (sizeof(E) == 4) {
                    v[a][c] = row[16 * c];
                } else {
                    v[a][c] = us2{row[16 * (2 * c)], row[16 * (2 * c + 1)]};
                }
            }
        }
        __syncthreads();
    } else {
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
    }
    D::template publish<0>(v, 0, lb, tx, ty);
    D::template steps<0>(v, tx, ty, lb);
    if constexpr (STAGE) {
        __syncthreads();  // every thread is done with the last block's slot
        for (int a = 0; a < D::RA; ++a) {
            FW_LDS E *row = lb + (ty + 16 * a) * B + tx;
            for (int b = 0; b < D::CW; ++b) row[16 * b] = lane_get<E>(v[a], b);
        }
        __syncthreads();
        constexpr int V = 16 / (int)sizeof(E);
        constexpr int VPR = B / V;
        dst = scalar_ptr(dst);
#pragma unroll 4
        for (int q = threadIdx.x; q < B * VPR; q += 256) {
            const int r = q / VPR, cv = q % VPR;
            const v4u32 x = *(const FW_LDS v4u32 *)(lb + r * B + cv * V);
            *retype<v4u32>(dst + (int64_t)r * ldd_ + cv * V) = x;
            if (dst2) {
                uint32_t *d2 = reinterpret_cast<uint32_t *>(dst2 + (int64_t)r * ldd2 + cv * V);
                __hip_atomic_store(d2 + 0, x.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(d2 + 1, x.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(d2 + 2, x.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(d2 + 3, x.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
        for (int a = 0; a < D::RA; ++a) {
            const auto row = dst + (int64_t)(ty + 16 * a) * ldd_ + tx;
            E *row2 = dst2 ? dst2 + (int64_t)(ty + 16 * a) * ldd2 + tx : nullptr;
            for (int b = 0; b < D::CW; ++b) {
                const E x = lane_get<E>(v[a], b);
                row[16 * b] = x;
                if (row2) __hip_atomic_store(row2 + 16 * b, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
}

template <typename E, int B, int S, bool STAGE, typename SrcP, typename DstP>
__device__ __attribute__((noinline)) void diag_close_call(SrcP src, int64_t lds_, DstP dst, int64_t ldd_,
                                                          E *__restrict__ dst2, int64_t ldd2, E *buf) {
    diag_close_body<E, B, S, STAGE>(src, lds_, dst, ldd_, dst2, ldd2, buf);
}

// LDS elements diag_close<E, B, S, STAGE> needs (16-byte aligned): the
// blocks' slots, and with STAGE the whole tile.
template <typename E, int B, int S = diag_steps<E, B>(), bool STAGE = false>
constexpr int diag_lds_elems() {
    return STAGE && B * B > Diag<E, B, S>::LDS_ELEMS ? B * B : Diag<E, B, S>::LDS_ELEMS;
}

// Close the B x B tile at src (row pitch lds_) and write it to dst, and to
// dst2 when given (with agent-scope stores: dst2 is a tile that other
// workgroups read); buf holds diag_lds_elems<E, B, S, STAGE>() elements of
// LDS.  With STAGE the tile moves between memory and registers through LDS
// as 16-byte vectors (src, dst and dst2 rows 16-byte aligned); without, each
// thread reads and writes its own strided elements.  Small tiles are
// inlined; the larger ones are a call of their own, so that their register
// demand is not added to the caller's.
template <typename E, int B, int S = diag_steps<E, B>(), bool STAGE = false, typename SrcP, typename DstP>
__device__ __attribute__((always_inline)) inline void diag_close(SrcP src, int64_t lds_, DstP dst, int64_t ldd_,
                                                            E *__restrict__ dst2, int64_t ldd2, E *buf) {
    if constexpr (B >= 128)
        diag_close_call<E, B, S, STAGE>(src, lds_, dst, ldd_, dst2, ldd2, buf);
    else
        diag_close_body<E, B, S, STAGE>(src, lds_, dst, ldd_, dst2, ldd2, buf);
}

}  // namespace fw
