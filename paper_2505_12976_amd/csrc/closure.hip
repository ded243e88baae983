// Widest-path closure p of the weighted tournament graph (Section 2.1), by
// the Floyd-Warshall recurrence p[i][j] = max(p[i][j], min(p[i][k], p[k][j]))
// (the classical algorithm of Section 5.2) in blocked form.
//
// The matrix is cut into B x B tiles.  Round r makes block r of vertices
// available as intermediates:
//   diag   the tile (r, r) is closed by the plain recurrence over its own
//          vertices (sequential in k, one workgroup);
//   panel  a tile (r, J) becomes max(P[r][J], D* (x) P[r][J]) and a tile
//          (I, r) becomes max(P[I][r], P[I][r] (x) D*), where D* is the closed
//          diagonal tile and (x) is the (max, min) product.  A widest path from
//          i in block r to j outside it that uses block r as intermediates
//          leaves the block for the last time at some k, so one product
//          with the closed diagonal tile is exact and has no sequential k;
//   rest   every other tile becomes max(P[I][J], P[I][r] (x) P[r][J]).
// All three are exact in integers, so the result does not depend on B or on
// the order in which independent tiles are processed.
//
// Main path: one persistent launch.  Every tile has a fixed owner workgroup
// (its state never leaves that workgroup's XCD).  An owner publishes the
// round-r diagonal and panel tiles into a write-once buffer (one slot per
// round and tile) and raises a flag; consumers wait on the flags they need.
// Each workgroup works through its tiles round by round -- diagonal, then
// panels, then the rest tiles that feed the next round's diagonal and panels,
// then the others -- so round r+1 starts while round r is still finishing.
// Every wait is on an item of an earlier (round, role) than the waiter's, and
// a cooperative launch keeps all workgroups resident, so every wait ends;
// a bounded spin turns anything else into a device error instead of a hang.
//
// uint16 matrices run two columns per 32-bit lane with v_pk_min_u16 and
// v_pk_max_u16 (one instruction per update); int32 matrices use v_min_i32
// and v_max3_i32 over pairs of k.  The matrix is padded with zero rows and
// columns to a multiple of B; padded vertices have no edges and change
// nothing.
#include "internal.h"

namespace {

typedef __attribute__((ext_vector_type(2))) unsigned short us2;

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

// ------------------------------------------------------------------ weights
// P[i][j] = edge weight from d (winning votes or margin); zero padding.
template <typename E>
__global__ __launch_bounds__(256) void k_weights(const E *__restrict__ d, int64_t ldd, int32_t m, int mode,
                                                 E *__restrict__ P, int64_t ld, int32_t mp) {
    __shared__ E a[64][65];
    __shared__ E b[64][65];
    const int32_t I0 = blockIdx.y * 64, J0 = blockIdx.x * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int32_t i = I0 + r, j = J0 + c;
        a[r][c] = (i < m && j < m) ? d[(int64_t)i * ldd + j] : (E)0;
        const int32_t i2 = J0 + r, j2 = I0 + c;  // block (J, I)
        b[r][c] = (i2 < m && j2 < m) ? d[(int64_t)i2 * ldd + j2] : (E)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int32_t i = I0 + r, j = J0 + c;
        if (i >= mp || j >= mp) continue;
        const E x = a[r][c], y = b[c][r];  // d[i][j], d[j][i]
        E w = 0;
        if (i != j && i < m && j < m && x > y) w = mode == SCHULZE_MARGIN ? (E)(x - y) : x;
        P[(int64_t)i * ld + j] = w;
    }
}

// p[i][j] = P[i][j] for i != j, 0 on the diagonal.
template <typename E>
__global__ __launch_bounds__(256) void k_fw_store(const E *__restrict__ P, int64_t ld, int32_t m, E *__restrict__ p,
                                                  int64_t ldp) {
    const int32_t col_blocks = (m + 255) / 256;
    const int32_t i = blockIdx.x / col_blocks;
    const int32_t j = (blockIdx.x % col_blocks) * 256 + threadIdx.x;
    if (j >= m) return;
    p[(int64_t)i * ldp + j] = i == j ? (E)0 : P[(int64_t)i * ld + j];
}

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

template <typename E>
__device__ inline void copy_block(E *__restrict__ dst, int dst_pitch, const E *__restrict__ src, int64_t src_pitch,
                                  int rows, int cols) {
    // cols * sizeof(E) is a multiple of 16; rows of src and dst are 16-byte aligned
    const int vpr = cols * (int)sizeof(E) / 16;
    for (int v = threadIdx.x; v < rows * vpr; v += 256) {
        const int rr = v / vpr, cv = v % vpr;
        const uint4 x = *reinterpret_cast<const uint4 *>(src + rr * src_pitch + cv * (16 / sizeof(E)));
        *reinterpret_cast<uint4 *>(dst + rr * dst_pitch + cv * (16 / sizeof(E))) = x;
    }
}

template <typename E, int B>
__device__ inline void acc_load(Acc<E, B> &a, const E *__restrict__ src, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int ii = 0; ii < C::TM; ++ii) {
        const W *row = reinterpret_cast<const W *>(src + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) a.c[ii][jj] = row[jj];
    }
}

template <typename E, int B>
__device__ inline void acc_store(const Acc<E, B> &a, E *__restrict__ dst, int64_t ld) {
    using C = Cfg<E, B>;
    using W = typename Lane<E>::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int ii = 0; ii < C::TM; ++ii) {
        W *row = reinterpret_cast<W *>(dst + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj) row[jj] = a.c[ii][jj];
    }
}

// a = max(a, A (x) Bm) with A, Bm B x B tiles in global memory (row pitches
// lda, ldb).  lds holds Cfg::LDS_ELEMS elements.  Starts and ends with a
// barrier, so A or Bm may be the tile that the caller overwrites afterwards.
template <typename E, int B>
__device__ inline void acc_product(Acc<E, B> &a, const E *__restrict__ A, int64_t lda, const E *__restrict__ Bm,
                                   int64_t ldb, E *lds) {
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

template <typename E, int B>
__device__ inline void diag_close(const E *__restrict__ src, int64_t lds_, E *__restrict__ dst, int64_t ldd_,
                                  E *__restrict__ dst2, int64_t ldd2, E *buf) {
    using D = Diag<E, B>;
    using W = typename D::W;
    E *rowbuf = buf;          // [2][B]: thread tx's columns at tx*CW ..
    E *colbuf = buf + 2 * B;  // [2][B]: thread ty's rows at ty*RA ..
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    W v[D::RA][D::WC];
    for (int a = 0; a < D::RA; ++a) {
        const E *row = src + (int64_t)(ty + 16 * a) * lds_ + tx;
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
        E *row = dst + (int64_t)(ty + 16 * a) * ldd_ + tx;
        E *row2 = dst2 ? dst2 + (int64_t)(ty + 16 * a) * ldd2 + tx : nullptr;
        for (int b = 0; b < D::CW; ++b) {
            const E x = lane_get<E>(v[a], b);
            row[16 * b] = x;
            if (row2) row2[16 * b] = x;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ persistent launch
template <typename E>
struct PersistArgs {
    E *P;               // padded matrix, pitch ld
    int64_t ld;
    int32_t nb;
    E *ring;            // nb rounds x (2 nb + 1) published tiles of B x B
    int32_t *flags;     // nb x (2 nb + 1), zero on entry
    int32_t *abort;     // zero on entry
    int32_t *err;       // device error word
    int64_t spin_limit; // polls before a wait is declared stuck
};

constexpr int MAX_OWNED = 512;

// Owner of tile (I, J): every block row and block column spreads over
// distinct workgroups (so the panels of a round are computed in parallel).
__device__ inline int32_t tile_owner(int32_t I, int32_t J, int32_t nb, int32_t G) {
    int32_t q = G / nb;
    if (q < 1) q = 1;
    return (((I + J) % nb) + nb * (I % q)) % G;
}

// slot of a published tile within a round: 0 diag, 1+J row panel, 1+nb+I column panel
__device__ inline int64_t slot_index(int32_t r, int32_t slot, int32_t nb) { return (int64_t)r * (2 * nb + 1) + slot; }

__device__ inline bool wait_flags(const int32_t *f0, const int32_t *f1, int32_t *abort, int64_t limit) {
    __shared__ int32_t ok;
    if (threadIdx.x == 0) {
        int32_t good = 1;
        int64_t spins = 0;
        const int32_t *fs[2] = {f0, f1};
        for (int q = 0; q < 2 && good; ++q) {
            if (!fs[q]) continue;
            while (__hip_atomic_load(fs[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > limit) {
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        ok = good;
    }
    __syncthreads();
    const bool res = ok != 0;
    __syncthreads();
    return res;
}

// Make this workgroup's stores of a published tile visible device-wide, then
// raise its flag.  Published slots are written once per launch and read only
// after their flag is seen, so no reader can hold an older copy of them.
__device__ inline void raise_flag(int32_t *f) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename E, int B>
__global__ __launch_bounds__(256, (sizeof(E) == 2 || B < 128) ? 2 : 1) void k_fw_persist(PersistArgs<E> a) {
    using C = Cfg<E, B>;
    __shared__ __attribute__((aligned(16))) E lds[C::LDS_ELEMS > 4 * B ? C::LDS_ELEMS : 4 * B];
    __shared__ int32_t owned[MAX_OWNED];
    __shared__ int32_t n_owned;
    const int32_t nb = a.nb, G = gridDim.x, w = blockIdx.x;
    const int64_t tile_elems = (int64_t)B * B;

    if (threadIdx.x == 0) n_owned = 0;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < nb * nb; t += 256) {
        if (tile_owner(t / nb, t % nb, nb, G) == w) {
            const int32_t q = atomicAdd(&n_owned, 1);
            if (q < MAX_OWNED) owned[q] = t;
        }
    }
    __syncthreads();
    const int32_t no = n_owned;
    if (no > MAX_OWNED) {  // the host sizes the grid so that this cannot happen
        if (threadIdx.x == 0) {
            set_device_error(a.err, SCHULZE_EDEVICE);
            __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }

    auto tileP = [&](int32_t I, int32_t J) { return a.P + (int64_t)I * B * a.ld + (int64_t)J * B; };
    auto ring = [&](int32_t r, int32_t slot) { return a.ring + slot_index(r, slot, nb) * tile_elems; };
    auto flag = [&](int32_t r, int32_t slot) { return a.flags + slot_index(r, slot, nb); };

    for (int32_t r = 0; r < nb; ++r) {
        // diagonal
        if (tile_owner(r, r, nb, G) == w) {
            diag_close<E, B>(tileP(r, r), a.ld, tileP(r, r), a.ld, ring(r, 0), B, lds);
            raise_flag(flag(r, 0));
        }
        // panels
        for (int32_t q = 0; q < no; ++q) {
            const int32_t I = owned[q] / nb, J = owned[q] % nb;
            if ((I == r) == (J == r)) continue;
            if (!wait_flags(flag(r, 0), nullptr, a.abort, a.spin_limit)) goto stuck;
            Acc<E, B> acc;
            acc_load<E, B>(acc, tileP(I, J), a.ld);
            int32_t slot;
            if (I == r) {  // row panel: D* (x) P[r][J]
                acc_product<E, B>(acc, ring(r, 0), B, tileP(I, J), a.ld, lds);
                slot = 1 + J;
            } else {       // column panel: P[I][r] (x) D*
                acc_product<E, B>(acc, tileP(I, J), a.ld, ring(r, 0), B, lds);
                slot = 1 + nb + I;
            }
            acc_store<E, B>(acc, tileP(I, J), a.ld);
            acc_store<E, B>(acc, ring(r, slot), B);
            raise_flag(flag(r, slot));
        }
        // rest tiles: those that feed round r+1's diagonal and panels first
        for (int pass = 0; pass < 2; ++pass) {
            for (int32_t q = 0; q < no; ++q) {
                const int32_t I = owned[q] / nb, J = owned[q] % nb;
                if (I == r || J == r) continue;
                const bool next = I == r + 1 || J == r + 1;
                if (next != (pass == 0)) continue;
                if (!wait_flags(flag(r, 1 + J), flag(r, 1 + nb + I), a.abort, a.spin_limit)) goto stuck;
                Acc<E, B> acc;
                acc_load<E, B>(acc, tileP(I, J), a.ld);
                acc_product<E, B>(acc, ring(r, 1 + nb + I), B, ring(r, 1 + J), B, lds);
                acc_store<E, B>(acc, tileP(I, J), a.ld);
            }
        }
    }
    return;
stuck:
    if (threadIdx.x == 0) set_device_error(a.err, SCHULZE_EDEVICE);
}

// ------------------------------------------------------------------ per-phase launches
// Used when a cooperative launch is not available: three launches per round.
template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_diag(E *__restrict__ P, int64_t ld, int32_t r) {
    __shared__ __attribute__((aligned(16))) E buf[4 * B];
    E *t = P + (int64_t)r * B * ld + (int64_t)r * B;
    diag_close<E, B>(t, ld, t, ld, nullptr, 0, buf);
}

template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_panel(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r) {
    __shared__ __attribute__((aligned(16))) E lds[Cfg<E, B>::LDS_ELEMS];
    const int32_t t = blockIdx.x;
    int32_t I, J;
    if (t < nb - 1) {
        I = r;
        J = t < r ? t : t + 1;
    } else {
        const int32_t u = t - (nb - 1);
        J = r;
        I = u < r ? u : u + 1;
    }
    E *Ct = P + (int64_t)I * B * ld + (int64_t)J * B;
    Acc<E, B> acc;
    acc_load<E, B>(acc, Ct, ld);
    acc_product<E, B>(acc, P + (int64_t)I * B * ld + (int64_t)r * B, ld, P + (int64_t)r * B * ld + (int64_t)J * B,
                      ld, lds);
    acc_store<E, B>(acc, Ct, ld);
}

template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_rest(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r) {
    __shared__ __attribute__((aligned(16))) E lds[Cfg<E, B>::LDS_ELEMS];
    const int32_t t = blockIdx.x;
    const int32_t i = t / (nb - 1), j = t % (nb - 1);
    const int32_t I = i < r ? i : i + 1, J = j < r ? j : j + 1;
    E *Ct = P + (int64_t)I * B * ld + (int64_t)J * B;
    Acc<E, B> acc;
    acc_load<E, B>(acc, Ct, ld);
    acc_product<E, B>(acc, P + (int64_t)I * B * ld + (int64_t)r * B, ld, P + (int64_t)r * B * ld + (int64_t)J * B,
                      ld, lds);
    acc_store<E, B>(acc, Ct, ld);
}

template <typename E, int B>
int run_closure(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, E *p, int64_t ldp) {
    const int32_t mp = (int32_t)round_up(m, B);
    const int32_t nb = mp / B;
    const int64_t ld = mp;
    int rc = ws_reserve(ctx, WS_CLOSURE, sizeof(E) * (size_t)mp * mp);
    if (rc != SCHULZE_OK) return rc;
    E *P = static_cast<E *>(ctx->ws[WS_CLOSURE]);
    dim3 wgrid((unsigned)ceil_div(mp, 64), (unsigned)ceil_div(mp, 64));
    SCHULZE_LAUNCH(ctx, K_WEIGHTS, s, k_weights<E><<<wgrid, dim3(256), 0, s>>>(d, ldd, m, mode, P, ld, mp));

    bool done = false;
    if (nb > 1 && !ctx->force_phased) {
        // persistent dataflow launch
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fw_persist<E, B>, 256, 0) != hipSuccess)
            per_cu = 0;
        int64_t G = (int64_t)per_cu * ctx->num_cus;
        if (G > (int64_t)nb * nb) G = (int64_t)nb * nb;
        const int64_t tiles_per_wg = ceil_div((int64_t)nb * nb, G > 0 ? G : 1);
        if (G >= 1 && tiles_per_wg <= MAX_OWNED) {
            const int64_t nslots = (int64_t)nb * (2 * nb + 1);
            const size_t ring_bytes = sizeof(E) * (size_t)nslots * B * B;
            const size_t flag_bytes = sizeof(int32_t) * (size_t)(nslots + 64);
            if ((rc = ws_reserve(ctx, WS_RING, ring_bytes)) != SCHULZE_OK) return rc;
            if ((rc = ws_reserve(ctx, WS_FLAGS, flag_bytes)) != SCHULZE_OK) return rc;
            int32_t *flags = static_cast<int32_t *>(ctx->ws[WS_FLAGS]);
            if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(flags), (size_t)(nslots + 64), 0u)) != SCHULZE_OK)
                return rc;
            PersistArgs<E> pa{P, ld, nb, static_cast<E *>(ctx->ws[WS_RING]), flags, flags + nslots, ctx->err,
                              (int64_t)1 << 22};
            void *args[] = {&pa};
            int tok;
            timing_begin(ctx, K_FW_PERSIST, s, &tok);
            hipError_t e = hipLaunchCooperativeKernel((const void *)k_fw_persist<E, B>, dim3((unsigned)G), dim3(256),
                                                      args, 0, s);
            timing_end(ctx, tok, s);
            if (e == hipSuccess) {
                done = true;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    if (!done) {
        for (int32_t r = 0; r < nb; ++r) {
            SCHULZE_LAUNCH(ctx, K_FW_DIAG, s, k_fw_diag<E, B><<<dim3(1), dim3(256), 0, s>>>(P, ld, r));
            if (nb > 1) {
                SCHULZE_LAUNCH(ctx, K_FW_PANEL, s,
                               k_fw_panel<E, B><<<dim3((unsigned)(2 * (nb - 1))), dim3(256), 0, s>>>(P, ld, nb, r));
                SCHULZE_LAUNCH(ctx, K_FW_REST, s,
                               k_fw_rest<E, B><<<dim3((unsigned)((nb - 1) * (nb - 1))), dim3(256), 0, s>>>(P, ld, nb,
                                                                                                           r));
            }
        }
    }
    dim3 sgrid((unsigned)(ceil_div(m, 256) * m));
    SCHULZE_LAUNCH(ctx, K_FW_STORE, s, k_fw_store<E><<<sgrid, dim3(256), 0, s>>>(P, ld, m, p, ldp));
    return SCHULZE_OK;
}

}  // namespace

extern "C" int schulze_closure(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m, int dtype,
                               int mode, void *p, int64_t ldp) {
    if (!ctx || !d || !p) return SCHULZE_EINVAL;
    if (m < 1 || ldd < m || ldp < m) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (m > 65535) return SCHULZE_EUNSUPPORTED;
    const size_t es = dtype == SCHULZE_U16 ? 2 : 4;
    {
        // p must not overlap d
        const char *d0 = static_cast<const char *>(d), *p0 = static_cast<const char *>(p);
        const char *d1 = d0 + es * (size_t)((m - 1) * ldd + m), *p1 = p0 + es * (size_t)((m - 1) * ldp + m);
        if (p0 < d1 && d0 < p1) return SCHULZE_EINVAL;
    }
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16)
        return run_closure<uint16_t, 64>(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode,
                                         static_cast<uint16_t *>(p), ldp);
    if (m >= 2048)
        return run_closure<int32_t, 128>(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode,
                                         static_cast<int32_t *>(p), ldp);
    return run_closure<int32_t, 64>(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode,
                                    static_cast<int32_t *>(p), ldp);
}
