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
// All three are exact in integers, so the result does not depend on B.
//
// uint16 matrices run two columns per 32-bit lane with v_pk_min_u16 and
// v_pk_max_u16 (one instruction per update); int32 matrices use v_min_i32
// and v_max3_i32 over pairs of k.  The matrix is padded with zero rows and
// columns to a multiple of B; padded vertices have no edges and change
// nothing.
#include "internal.h"

namespace {

typedef __attribute__((ext_vector_type(2))) unsigned short us2;

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

// ------------------------------------------------------------------ diag
template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_diag(E *__restrict__ P, int64_t ld, int32_t r) {
    __shared__ E t[B][B];  // row-wise thread mapping: no bank conflicts
    E *base = P + (int64_t)r * B * ld + (int64_t)r * B;
    for (int e = threadIdx.x; e < B * B; e += 256) t[e / B][e % B] = base[(int64_t)(e / B) * ld + e % B];
    for (int k = 0; k < B; ++k) {
        __syncthreads();
        // row k and column k do not change in step k
        for (int e = threadIdx.x; e < B * B; e += 256) {
            const int i = e / B, j = e % B;
            const E via = min(t[i][k], t[k][j]);
            if (via > t[i][j]) t[i][j] = via;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < B * B; e += 256) base[(int64_t)(e / B) * ld + e % B] = t[e / B][e % B];
}

// ------------------------------------------------------------------ product
// C = max(C, A (x) Bm) for one B x B tile, A = P[I][r], Bm = P[r][J],
// C = P[I][J].  256 threads as 16 x 16; each owns TM rows (ty*TM ..) and TN
// columns (tx*TN ..).  k is staged through LDS in chunks of KC.
template <typename E, int B>
struct ProdCfg {
    static constexpr int TM = B / 16;
    static constexpr int TN = B / 16;
    static constexpr int KC = 32;
    static constexpr int PADA = 16 / sizeof(E);  // keep 16-byte row alignment
    static constexpr int PADB = 16 / sizeof(E);
};

template <typename E>
__device__ inline void copy_block(E *__restrict__ dst, int dst_pitch, const E *__restrict__ src, int64_t src_pitch,
                                  int rows, int cols) {
    // cols * sizeof(E) is a multiple of 16
    const int vpr = cols * (int)sizeof(E) / 16;
    for (int v = threadIdx.x; v < rows * vpr; v += 256) {
        const int rr = v / vpr, cv = v % vpr;
        const uint4 x = *reinterpret_cast<const uint4 *>(src + rr * src_pitch + cv * (16 / sizeof(E)));
        *reinterpret_cast<uint4 *>(dst + rr * dst_pitch + cv * (16 / sizeof(E))) = x;
    }
}

template <typename E, int B>
__device__ inline void tile_product(E *__restrict__ P, int64_t ld, int32_t I, int32_t J, int32_t r) {
    using C = ProdCfg<E, B>;
    constexpr int TM = C::TM, TN = C::TN, KC = C::KC;
    constexpr int LA = KC + C::PADA, LB = B + C::PADB;
    __shared__ __attribute__((aligned(16))) E As[B * LA];
    __shared__ __attribute__((aligned(16))) E Bs[KC * LB];

    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    E *Cg = P + (int64_t)I * B * ld + (int64_t)J * B;
    const E *Ag = P + (int64_t)I * B * ld + (int64_t)r * B;
    const E *Bg = P + (int64_t)r * B * ld + (int64_t)J * B;

    if constexpr (sizeof(E) == 4) {
        E c[TM][TN];
        for (int ii = 0; ii < TM; ++ii) {
            const E *row = Cg + (int64_t)(ty * TM + ii) * ld + tx * TN;
            for (int jj = 0; jj < TN; ++jj) c[ii][jj] = row[jj];
        }
        for (int kc = 0; kc < B; kc += KC) {
            __syncthreads();
            copy_block<E>(As, LA, Ag + kc, ld, B, KC);
            copy_block<E>(Bs, LB, Bg + (int64_t)kc * ld, ld, KC, B);
            __syncthreads();
#pragma unroll 2
            for (int k = 0; k < KC; k += 2) {
                E a0[TM], a1[TM], b0[TN], b1[TN];
                for (int ii = 0; ii < TM; ++ii) {
                    a0[ii] = As[(ty * TM + ii) * LA + k];
                    a1[ii] = As[(ty * TM + ii) * LA + k + 1];
                }
                for (int jj = 0; jj < TN; ++jj) {
                    b0[jj] = Bs[k * LB + tx * TN + jj];
                    b1[jj] = Bs[(k + 1) * LB + tx * TN + jj];
                }
                for (int ii = 0; ii < TM; ++ii)
                    for (int jj = 0; jj < TN; ++jj)
                        c[ii][jj] = max(c[ii][jj], max(min(a0[ii], b0[jj]), min(a1[ii], b1[jj])));
            }
        }
        for (int ii = 0; ii < TM; ++ii) {
            E *row = Cg + (int64_t)(ty * TM + ii) * ld + tx * TN;
            for (int jj = 0; jj < TN; ++jj) row[jj] = c[ii][jj];
        }
    } else {
        // two uint16 columns per 32-bit lane
        constexpr int WN = TN / 2;
        us2 c[TM][WN];
        for (int ii = 0; ii < TM; ++ii) {
            const us2 *row = reinterpret_cast<const us2 *>(Cg + (int64_t)(ty * TM + ii) * ld + tx * TN);
            for (int jj = 0; jj < WN; ++jj) c[ii][jj] = row[jj];
        }
        for (int kc = 0; kc < B; kc += KC) {
            __syncthreads();
            copy_block<E>(As, LA, Ag + kc, ld, B, KC);
            copy_block<E>(Bs, LB, Bg + (int64_t)kc * ld, ld, KC, B);
            __syncthreads();
#pragma unroll 4
            for (int k = 0; k < KC; ++k) {
                us2 bp[WN];
                for (int jj = 0; jj < WN; ++jj)
                    bp[jj] = *reinterpret_cast<const us2 *>(&Bs[k * LB + tx * TN + 2 * jj]);
                for (int ii = 0; ii < TM; ++ii) {
                    const unsigned short av = As[(ty * TM + ii) * LA + k];
                    const us2 aa = {av, av};
                    for (int jj = 0; jj < WN; ++jj)
                        c[ii][jj] = __builtin_elementwise_max(c[ii][jj], __builtin_elementwise_min(aa, bp[jj]));
                }
            }
        }
        for (int ii = 0; ii < TM; ++ii) {
            us2 *row = reinterpret_cast<us2 *>(Cg + (int64_t)(ty * TM + ii) * ld + tx * TN);
            for (int jj = 0; jj < WN; ++jj) row[jj] = c[ii][jj];
        }
    }
}

// Panel phase: tiles (r, J) for J != r, then (I, r) for I != r.
template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_panel(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r) {
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
    tile_product<E, B>(P, ld, I, J, r);
}

// Remaining tiles (I, J), I != r, J != r.
template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_rest(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r) {
    const int32_t t = blockIdx.x;
    const int32_t i = t / (nb - 1), j = t % (nb - 1);
    const int32_t I = i < r ? i : i + 1, J = j < r ? j : j + 1;
    tile_product<E, B>(P, ld, I, J, r);
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
    for (int32_t r = 0; r < nb; ++r) {
        SCHULZE_LAUNCH(ctx, K_FW_DIAG, s, k_fw_diag<E, B><<<dim3(1), dim3(256), 0, s>>>(P, ld, r));
        if (nb > 1) {
            SCHULZE_LAUNCH(ctx, K_FW_PANEL, s,
                           k_fw_panel<E, B><<<dim3((unsigned)(2 * (nb - 1))), dim3(256), 0, s>>>(P, ld, nb, r));
            SCHULZE_LAUNCH(ctx, K_FW_REST, s,
                           k_fw_rest<E, B><<<dim3((unsigned)((nb - 1) * (nb - 1))), dim3(256), 0, s>>>(P, ld, nb, r));
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
