// Pairwise preference counts d[x][y] (Section 2.1: profile of weak orders).
//
// d[x][y] is the total weight of voters who list x and list y later or not
// at all.  Ballots take one of two routes:
//
//  * full rankings (at least m-1 listed candidates): the rank of every
//    candidate is scattered into a position array, two voters per 32-bit
//    word (low half: voter 2q, high half: voter 2q+1).  For one (x, y) pair
//    and one voter, the 16-bit difference t = (pos(x) - pos(y)) mod 2^16
//    equals pos(x) - pos(y) + 2^16 [pos(x) < pos(y)].  Summed over voters,
//        sum t = Sx - Sy + 2^16 * #(x before y),
//    where Sx is the sum of x's positions.  One v_pk_sub_u16 yields t for two
//    voters and one v_dot2_u32_u16 adds both halves into a 32-bit
//    accumulator, so each comparison costs one VALU lane-op; the count is
//    recovered as (acc - Sx + Sy) >> 16, exact while fewer than 2^16 voters
//    are summed at once.  Full rankings have no ties, so only tiles with
//    x-block <= y-block are computed and d[y][x] = voters - d[x][y].
//
//  * truncated ballots: d[x][y] = R[x] - C[y][x], where R[x] is the weight of
//    ballots listing x and C[y][x] the weight of ballots listing y before x;
//    the listed pairs are scattered with atomics.
//
// Both routes accumulate into one m x m uint32 matrix that a final pass adds
// to R and converts to the output dtype.
#include "internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int CT = 128;         // count tile (candidates per side)
constexpr int VC = 32;          // voter pairs per staged chunk
constexpr int CNT_THREADS = 256;
constexpr int SEG_PAIRS = 32767; // at most 65534 voters per exact segment
constexpr int SEGC = SEG_PAIRS / VC;
constexpr int SCATTER_CH = 8192; // candidates per LDS chunk of the scatter

// Workspace layout of WS_BALLOT_META (int32 words).
struct Meta {
    int32_t *counters;  // [0] = number of full rankings
    int32_t *len;       // listed length per ballot
    int32_t *full_src;  // slot -> ballot index for full rankings
};

__device__ inline int32_t read_id(const void *ballots, int dtype32, int64_t idx) {
    if (dtype32) {
        int32_t v = static_cast<const int32_t *>(ballots)[idx];
        return v < 0 ? -1 : v;
    }
    uint16_t v = static_cast<const uint16_t *>(ballots)[idx];
    return v == 0xFFFF ? -1 : (int32_t)v;
}

// ------------------------------------------------------------------ scan
// One workgroup per ballot: listed length, id range and duplicate checks
// (LDS bitmap over candidates), and the full/truncated split.
__global__ __launch_bounds__(SCAN_THREADS) void k_ballot_scan(const void *__restrict__ ballots, int dtype32,
                                                              int64_t n, int32_t L, int32_t m, Meta meta,
                                                              int32_t *err) {
    extern __shared__ uint32_t seen[];  // ceil(m/32) words
    __shared__ int32_t first_pad;
    const int64_t v = blockIdx.x;
    if (v >= n) return;
    const int words = (m + 31) >> 5;
    for (int i = threadIdx.x; i < words; i += SCAN_THREADS) seen[i] = 0u;
    if (threadIdx.x == 0) first_pad = L;
    __syncthreads();
    const int64_t base = v * (int64_t)L;
    for (int t = threadIdx.x; t < L; t += SCAN_THREADS)
        if (read_id(ballots, dtype32, base + t) < 0) atomicMin(&first_pad, t);
    __syncthreads();
    const int k = first_pad;
    bool bad = false;
    for (int t = threadIdx.x; t < k; t += SCAN_THREADS) {
        int32_t c = read_id(ballots, dtype32, base + t);
        if (c >= m) {
            bad = true;
            continue;
        }
        uint32_t bit = 1u << (c & 31);
        uint32_t old = atomicOr(&seen[c >> 5], bit);
        if (old & bit) bad = true;
    }
    if (bad) set_device_error(err, SCHULZE_EBALLOT);
    if (threadIdx.x == 0) {
        meta.len[v] = k;
        if (k >= m - 1) {
            int32_t slot = atomicAdd(&meta.counters[0], 1);
            meta.full_src[slot] = (int32_t)v;
        }
    }
}

// Short rows (L <= 64): one wavefront per ballot, one lane per entry.
__global__ __launch_bounds__(SCAN_THREADS) void k_ballot_scan_short(const void *__restrict__ ballots, int dtype32,
                                                                    int64_t n, int32_t L, int32_t m, Meta meta,
                                                                    int32_t *err) {
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * (SCAN_THREADS / 64) + (threadIdx.x >> 6);
    if (v >= n) return;
    const int64_t base = v * (int64_t)L;
    int32_t c = lane < L ? read_id(ballots, dtype32, base + lane) : -1;
    uint64_t pad = __ballot(c < 0);
    const int k = pad ? (int)__builtin_ctzll(pad) : 64;  // pad bit is set for every lane >= L
    bool listed = lane < k;
    bool bad = listed && c >= m;
    // duplicate check: compare with every earlier listed entry
    for (int j = 0; j < 64; ++j) {
        int32_t cj = __shfl(c, j);
        if (j < lane && listed && cj == c) bad = true;
    }
    if (__ballot(bad)) {
        if (lane == 0) set_device_error(err, SCHULZE_EBALLOT);
    }
    if (lane == 0) {
        meta.len[v] = k;
        if (k >= m - 1) {
            int32_t slot = atomicAdd(&meta.counters[0], 1);
            meta.full_src[slot] = (int32_t)v;
        }
    }
}

// ------------------------------------------------------------------ scatter
// One workgroup per voter pair q: positions of voters full_src[2q] (low
// half) and full_src[2q+1] (high half, or 0 for the missing partner of an
// odd count) for every candidate, in chunks of SCATTER_CH candidates staged
// in LDS, written as rows of `pitch` words (columns >= m are 0).
__global__ __launch_bounds__(256) void k_ballot_scatter(const void *__restrict__ ballots, int dtype32, int32_t L,
                                                        int32_t m, int32_t pitch, Meta meta,
                                                        uint32_t *__restrict__ pos) {
    __shared__ uint16_t buf[2 * SCATTER_CH];
    const int32_t n_full = meta.counters[0];
    const int64_t q = blockIdx.x;
    if (2 * q >= n_full) return;
    const bool has_hi = 2 * q + 1 < n_full;
    const int32_t src[2] = {meta.full_src[2 * q], has_hi ? meta.full_src[2 * q + 1] : -1};
    for (int32_t c0 = 0; c0 < pitch; c0 += SCATTER_CH) {
        const int32_t cn = min(SCATTER_CH, pitch - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += 256) {
            const int32_t c = c0 + i;
            // a ballot listing m-1 candidates leaves one unlisted: it is last
            buf[2 * i] = c < m ? (uint16_t)(m - 1) : (uint16_t)0;
            buf[2 * i + 1] = (c < m && has_hi) ? (uint16_t)(m - 1) : (uint16_t)0;
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            if (src[h] < 0) continue;
            const int32_t k = meta.len[src[h]];
            const int64_t base = (int64_t)src[h] * L;
            for (int t = threadIdx.x; t < k; t += 256) {
                const int32_t c = read_id(ballots, dtype32, base + t);
                if (c >= c0 && c < c0 + cn) buf[2 * (c - c0) + h] = (uint16_t)t;
            }
        }
        __syncthreads();
        const uint32_t *b32 = reinterpret_cast<const uint32_t *>(buf);
        for (int i = threadIdx.x; i < cn; i += 256) pos[q * (int64_t)pitch + c0 + i] = b32[i];
    }
}

// ------------------------------------------------------------------ dense count
// Persistent kernel.  Work units are (tile, chunk of VC voter pairs) with
// tiles (X, Y), X <= Y, over CT x CT candidate blocks; each workgroup takes a
// contiguous range of units (so every workgroup does the same amount of
// work) and flushes its accumulators into acc32 whenever the tile changes,
// a segment of SEG_PAIRS pairs ends, or its range ends.
struct DenseArgs {
    const uint32_t *pos;
    int32_t pitch;         // words per position row (multiple of CT)
    int32_t m;
    const int32_t *counters;
    uint32_t *acc;         // m x m
    int64_t lda;
};

__device__ inline void tile_coords(int32_t t, int32_t nb, int32_t &X, int32_t &Y) {
    int32_t x = 0, start = 0;
    while (start + (nb - x) <= t) {
        start += nb - x;
        ++x;
    }
    X = x;
    Y = x + (t - start);
}

__global__ __launch_bounds__(CNT_THREADS, 2) void k_count_dense(DenseArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t xs[VC][CT];
    __shared__ __attribute__((aligned(16))) uint32_t ys[VC][CT];
    __shared__ uint32_t sred[4][2 * CT];

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int32_t n_full = a.counters[0];
    const int64_t n_pairs = (n_full + 1) / 2;
    if (n_pairs == 0) return;
    const int32_t nb = a.pitch / CT;
    const int64_t ntiles = (int64_t)nb * (nb + 1) / 2;
    const int64_t cpt = (n_pairs + VC - 1) / VC;  // chunks per tile
    const int64_t U = ntiles * cpt;
    const int64_t u0 = U * blockIdx.x / gridDim.x;
    const int64_t u1 = U * (blockIdx.x + 1) / gridDim.x;
    if (u0 >= u1) return;

    // staging role: fixed 4 columns, pairs (tid >> 6) + 4 * q
    const int col4 = tid & 63;
    const int prow = tid >> 6;

    uint32_t acc[8][8];
    uint32_t s4[4];
    uint4 stage[8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) acc[i][j] = 0u;
    for (int e = 0; e < 4; ++e) s4[e] = 0u;

    int32_t cur_tile = -1, X = 0, Y = 0;
    int64_t seg_p0 = 0, seg_p1 = 0;

    auto load_unit = [&](int64_t u, uint4 (&dst)[8]) {
        const int32_t t = (int32_t)(u / cpt);
        const int64_t chunk = u % cpt;
        int32_t tX, tY;
        tile_coords(t, nb, tX, tY);
        const int32_t col = col4 < 32 ? tX * CT + col4 * 4 : tY * CT + (col4 - 32) * 4;
        const int64_t p0 = chunk * VC;
        for (int q = 0; q < 8; ++q) {
            const int64_t pr = p0 + prow + 4 * q;
            if (pr < n_pairs)
                dst[q] = *reinterpret_cast<const uint4 *>(a.pos + pr * a.pitch + col);
            else
                dst[q] = make_uint4(0u, 0u, 0u, 0u);
        }
    };

    auto flush = [&]() {
        __syncthreads();
        for (int e = 0; e < 4; ++e) sred[prow][col4 * 4 + e] = s4[e];
        __syncthreads();
        uint32_t sx[8], sy[8];
        for (int i = 0; i < 8; ++i) {
            const int c = ty * 8 + i;
            sx[i] = sred[0][c] + sred[1][c] + sred[2][c] + sred[3][c];
        }
        for (int j = 0; j < 8; ++j) {
            const int c = CT + tx * 8 + j;
            sy[j] = sred[0][c] + sred[1][c] + sred[2][c] + sred[3][c];
        }
        const int64_t hi = min((int64_t)n_full, 2 * seg_p1);
        const uint32_t nv = (uint32_t)max((int64_t)0, hi - 2 * seg_p0);
        for (int i = 0; i < 8; ++i) {
            const int32_t x = X * CT + ty * 8 + i;
            for (int j = 0; j < 8; ++j) {
                const int32_t y = Y * CT + tx * 8 + j;
                const uint32_t cnt = (acc[i][j] - sx[i] + sy[j]) >> 16;
                if (x < a.m && y < a.m && x != y) {
                    atomicAdd(&a.acc[(int64_t)x * a.lda + y], cnt);
                    if (X != Y) atomicAdd(&a.acc[(int64_t)y * a.lda + x], nv - cnt);
                }
                acc[i][j] = 0u;
            }
        }
        for (int e = 0; e < 4; ++e) s4[e] = 0u;
    };

    load_unit(u0, stage);
    for (int64_t u = u0; u < u1; ++u) {
        const int32_t t = (int32_t)(u / cpt);
        const int64_t chunk = u % cpt;
        if (t != cur_tile) {
            cur_tile = t;
            tile_coords(t, nb, X, Y);
            seg_p0 = chunk * VC;
        } else if (chunk % SEGC == 0) {
            seg_p0 = chunk * VC;
        }
        seg_p1 = min(n_pairs, (chunk + 1) * VC);

        __syncthreads();  // previous compute done with xs/ys
        for (int q = 0; q < 8; ++q) {
            const int pr = prow + 4 * q;
            uint32_t *dst = col4 < 32 ? &xs[pr][col4 * 4] : &ys[pr][(col4 - 32) * 4];
            *reinterpret_cast<uint4 *>(dst) = stage[q];
            s4[0] = __builtin_amdgcn_udot2(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, stage[q].x),
                                           (__attribute__((ext_vector_type(2))) unsigned short){1, 1}, s4[0], false);
            s4[1] = __builtin_amdgcn_udot2(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, stage[q].y),
                                           (__attribute__((ext_vector_type(2))) unsigned short){1, 1}, s4[1], false);
            s4[2] = __builtin_amdgcn_udot2(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, stage[q].z),
                                           (__attribute__((ext_vector_type(2))) unsigned short){1, 1}, s4[2], false);
            s4[3] = __builtin_amdgcn_udot2(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, stage[q].w),
                                           (__attribute__((ext_vector_type(2))) unsigned short){1, 1}, s4[3], false);
        }
        __syncthreads();
        if (u + 1 < u1) load_unit(u + 1, stage);  // overlaps the compute below

        typedef __attribute__((ext_vector_type(2))) unsigned short us2;
        const us2 ones = {1, 1};
#pragma unroll 1
        for (int v = 0; v < VC; ++v) {
            const uint4 xa = *reinterpret_cast<const uint4 *>(&xs[v][ty * 8]);
            const uint4 xb = *reinterpret_cast<const uint4 *>(&xs[v][ty * 8 + 4]);
            const uint4 ya = *reinterpret_cast<const uint4 *>(&ys[v][tx * 8]);
            const uint4 yb = *reinterpret_cast<const uint4 *>(&ys[v][tx * 8 + 4]);
            const uint32_t xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
            const uint32_t yv[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const us2 xi = __builtin_bit_cast(us2, xv[i]);
                us2 diff[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) diff[j] = xi - __builtin_bit_cast(us2, yv[j]);
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_udot2(diff[j], ones, acc[i][j], false);
            }
        }

        const bool last = u + 1 >= u1;
        bool boundary = last;
        if (!last) {
            const int32_t tn = (int32_t)((u + 1) / cpt);
            const int64_t cn = (u + 1) % cpt;
            boundary = tn != t || cn % SEGC == 0;
        }
        if (boundary) flush();
    }
}

// ------------------------------------------------------------------ sparse count
// One wavefront per truncated ballot: lane t handles listed entry t.  For
// every earlier entry i < t the pair (c_i before c_t) adds the voter's
// weight to C[c_i][c_t], i.e. subtracts it from acc[c_t][c_i]; every listed
// entry adds the weight to R.
__global__ __launch_bounds__(256) void k_count_sparse(const void *__restrict__ ballots, int dtype32, int64_t n,
                                                      int32_t L, int32_t m, const uint32_t *__restrict__ weight,
                                                      Meta meta, uint32_t *__restrict__ acc, int64_t lda,
                                                      uint32_t *__restrict__ rsum) {
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    const int32_t k = meta.len[v];
    if (k >= m - 1) return;  // full ranking: dense route
    const uint32_t w = weight ? weight[v] : 1u;
    if (w == 0u) return;
    const int64_t base = v * (int64_t)L;
    for (int t = lane; t < k; t += 64) {
        const int32_t ct = read_id(ballots, dtype32, base + t);
        if (ct >= m) continue;  // reported by the scan
        atomicAdd(&rsum[ct], w);
        uint32_t *row = acc + (int64_t)ct * lda;
        for (int i = 0; i < t; ++i) {
            const int32_t ci = read_id(ballots, dtype32, base + i);
            if (ci < m) atomicSub(&row[ci], w);
        }
    }
}

// ------------------------------------------------------------------ weighted dense count
// Full rankings with voter weights: plain compare-and-add per voter (the
// modular trick needs unit weights to bound the segment's total).
__global__ __launch_bounds__(256) void k_count_dense_weighted(const void *__restrict__ ballots, int dtype32,
                                                              int32_t L, int32_t m, const uint32_t *__restrict__ weight,
                                                              Meta meta, const uint32_t *__restrict__ pos,
                                                              int32_t pitch, uint32_t *__restrict__ acc, int64_t lda) {
    // one thread per (x, y) pair of a 16 x 16 block, looping over voters
    const int32_t x = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int32_t y = blockIdx.x * 16 + (threadIdx.x & 15);
    const int32_t n_full = meta.counters[0];
    if (x >= m || y >= m || x == y) return;
    uint32_t s = 0u;
    for (int32_t q = 0; 2 * q < n_full; ++q) {
        const uint32_t px = pos[(int64_t)q * pitch + x], py = pos[(int64_t)q * pitch + y];
        const uint32_t w0 = weight[meta.full_src[2 * q]];
        const uint32_t w1 = 2 * q + 1 < n_full ? weight[meta.full_src[2 * q + 1]] : 0u;
        s += ((px & 0xFFFFu) < (py & 0xFFFFu)) ? w0 : 0u;
        s += ((px >> 16) < (py >> 16)) ? w1 : 0u;
    }
    acc[(int64_t)x * lda + y] += s;
}

// ------------------------------------------------------------------ finish
// d[x][y] = acc[x][y] + R[x] for x != y, d[x][x] = 0; range-checked store.
template <typename T>
__global__ __launch_bounds__(256) void k_count_finish(const uint32_t *__restrict__ acc, int64_t lda,
                                                      const uint32_t *__restrict__ rsum, int32_t m, T *__restrict__ d,
                                                      int64_t ldd, uint32_t limit, int32_t *err) {
    const int32_t col_blocks = (m + 255) / 256;
    const int32_t x = blockIdx.x / col_blocks;
    const int32_t y = (blockIdx.x % col_blocks) * 256 + threadIdx.x;
    if (y >= m) return;
    uint32_t v = 0u;
    if (x != y) v = acc[(int64_t)x * lda + y] + rsum[x];
    if (v > limit) {
        set_device_error(err, SCHULZE_ERANGE);
        v = limit;
    }
    d[(int64_t)x * ldd + y] = (T)v;
}

}  // namespace

extern "C" int schulze_pairwise(schulze_ctx *ctx, void *stream, const void *ballots, int ballot_dtype, int64_t n,
                                int32_t L, int32_t m, const uint32_t *voter_weight, int d_dtype, void *d,
                                int64_t ldd) {
    if (!ctx || !d) return SCHULZE_EINVAL;
    if (ballot_dtype != SCHULZE_U16 && ballot_dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (d_dtype != SCHULZE_U16 && d_dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (n < 0 || m < 1 || m > 65535 || L < 1 || L > m || ldd < m) return SCHULZE_EINVAL;
    if (n > 0 && !ballots) return SCHULZE_EINVAL;
    if (n > (int64_t)INT32_MAX) return SCHULZE_EUNSUPPORTED;
    if (d_dtype == SCHULZE_U16 && !voter_weight && n > 65535) return SCHULZE_ERANGE;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int dtype32 = ballot_dtype == SCHULZE_I32;
    const int32_t pitch = (int32_t)round_up(m, CT);

    int rc;
    if ((rc = ws_reserve(ctx, WS_BALLOT_META, sizeof(int32_t) * (size_t)(64 + 2 * n))) != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_ACC32, sizeof(uint32_t) * (size_t)m * m)) != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_ROWSUM, sizeof(uint32_t) * (size_t)m)) != SCHULZE_OK) return rc;
    const int64_t max_pairs = (n + 1) / 2;
    const bool may_have_full = L >= m - 1 && n > 0;
    if (may_have_full &&
        (rc = ws_reserve(ctx, WS_POSITIONS, sizeof(uint32_t) * (size_t)max_pairs * pitch)) != SCHULZE_OK)
        return rc;

    int32_t *mw = static_cast<int32_t *>(ctx->ws[WS_BALLOT_META]);
    Meta meta{mw, mw + 64, mw + 64 + n};
    uint32_t *acc = static_cast<uint32_t *>(ctx->ws[WS_ACC32]);
    uint32_t *rsum = static_cast<uint32_t *>(ctx->ws[WS_ROWSUM]);
    uint32_t *pos = static_cast<uint32_t *>(ctx->ws[WS_POSITIONS]);
    const int64_t lda = m;

    if ((rc = fill_u32(ctx, s, (uint32_t *)meta.counters, 64, 0u)) != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, acc, (size_t)m * m, 0u)) != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, rsum, (size_t)m, 0u)) != SCHULZE_OK) return rc;

    if (n > 0) {
        if (L <= 64) {
            SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                           k_ballot_scan_short<<<dim3((unsigned)ceil_div(n, SCAN_THREADS / 64)), dim3(SCAN_THREADS),
                                                 0, s>>>(ballots, dtype32, n, L, m, meta, ctx->err));
        } else {
            const size_t lds = sizeof(uint32_t) * (size_t)((m + 31) / 32);
            SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                           k_ballot_scan<<<dim3((unsigned)n), dim3(SCAN_THREADS), lds, s>>>(ballots, dtype32, n, L,
                                                                                           m, meta, ctx->err));
        }
        // full rankings (only possible when L >= m - 1)
        if (may_have_full) {
            SCHULZE_LAUNCH(ctx, K_BALLOT_SCATTER, s,
                           k_ballot_scatter<<<dim3((unsigned)max_pairs), dim3(256), 0, s>>>(ballots, dtype32, L, m,
                                                                                           pitch, meta, pos));
            if (!voter_weight) {
                DenseArgs da{pos, pitch, m, meta.counters, acc, lda};
                const unsigned grid = (unsigned)ctx->num_cus * 2;
                SCHULZE_LAUNCH(ctx, K_COUNT_DENSE, s, k_count_dense<<<dim3(grid), dim3(CNT_THREADS), 0, s>>>(da));
            } else {
                dim3 grid((unsigned)ceil_div(m, 16), (unsigned)ceil_div(m, 16));
                SCHULZE_LAUNCH(ctx, K_COUNT_DENSE, s,
                               k_count_dense_weighted<<<grid, dim3(256), 0, s>>>(ballots, dtype32, L, m, voter_weight,
                                                                                 meta, pos, pitch, acc, lda));
            }
        }
        SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                       k_count_sparse<<<dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s>>>(
                           ballots, dtype32, n, L, m, voter_weight, meta, acc, lda, rsum));
    }
    dim3 fgrid((unsigned)(ceil_div(m, 256) * m));
    if (d_dtype == SCHULZE_U16) {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       k_count_finish<uint16_t><<<fgrid, dim3(256), 0, s>>>(acc, lda, rsum, m, (uint16_t *)d, ldd,
                                                                            65535u, ctx->err));
    } else {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       k_count_finish<int32_t><<<fgrid, dim3(256), 0, s>>>(acc, lda, rsum, m, (int32_t *)d, ldd,
                                                                           (uint32_t)INT32_MAX, ctx->err));
    }
    return SCHULZE_OK;
}
