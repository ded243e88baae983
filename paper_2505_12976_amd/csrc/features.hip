// Per-candidate features of the weighted tournament graph, the input of the
// learned winner proposer.  All are read off the pairwise counts d in one
// pass that reads every block of d once (a workgroup takes a pair of
// blocks and its transpose, see k_feature_rows):
//   0  Copeland score: #{y : d[x][y] > d[y][x]} / (m-1)
//   1  ties: #{y != x : d[x][y] = d[y][x]} / (m-1)
//   2  Borda score: sum_y d[x][y] / ((m-1) n)   (the order Section 4 uses for vertex ids)
//   3  largest outgoing edge weight / n
//   4  largest incoming edge weight / n
//   5  initialisation filter of Section 4: 1 if the largest incoming weight
//      exceeds the largest outgoing one (then x is never a winner)
//   6  mean outgoing weight / n      7  mean incoming weight / n
//   8  smallest margin d[x][y]-d[y][x] / n   9  largest margin / n
//   10 log(m) / 10
//   11 Copeland / max Copeland       12 Borda / max Borda
//   13 largest outgoing weight / its maximum over candidates
//   14 (largest outgoing - largest incoming weight) / n
//   15 1 (bias input)
// n is the number of voters (any positive scale works; it keeps features O(1)).
#include "internal.h"
#include "tile_io.h"

namespace {

constexpr int NF = 16;
// Lanes that share a row of a 64 x 64 tile; a thread takes RPT rows,
// r + h * ROW_STEP.  Four lanes and one row per thread: fewer shuffles per
// row reduction than eight lanes and two rows (1.01 ms instead of 1.28 ms
// at m = 32768, int32).
constexpr int ROW_LANES = 4;
constexpr int RPT = ROW_LANES * tio::T / 256;
constexpr int ROW_STEP = tio::T / RPT;

// Per-candidate statistics: one entry per candidate, or per candidate and
// column super-block for the partials.  Counts are non-negative and below
// 2^31, so every margin d[x][y] - d[y][x] fits in 32 bits.
struct RawStats {
    int32_t *cope, *ties, *max_out, *max_in, *min_marg, *max_marg;
    unsigned long long *borda, *sum_out, *sum_in;
};

// Sums over the columns of one workgroup (at most 4 tiles of 64): 32 bits
// hold them for 16-bit counts, int32 counts take 64.
template <typename E>
struct SumOf {
    using type = unsigned long long;
};
template <>
struct SumOf<uint16_t> {
    using type = uint32_t;
};

// Statistics of one candidate over a set of columns.
template <typename E>
struct Acc {
    using S = typename SumOf<E>::type;
    int32_t cope, ties, mx_out, mx_in, mn, mx;
    S borda, s_out, s_in;

    __device__ void init() {
        cope = ties = mx_out = mx_in = 0;
        mn = INT32_MAX;
        mx = INT32_MIN;
        borda = s_out = s_in = 0;
    }
    __device__ void merge(const Acc &o) {
        cope += o.cope;
        ties += o.ties;
        borda += o.borda;
        s_out += o.s_out;
        s_in += o.s_in;
        mx_out = max(mx_out, o.mx_out);
        mx_in = max(mx_in, o.mx_in);
        mn = min(mn, o.mn);
        mx = max(mx, o.mx);
    }
    // Combine the ROW_LANES adjacent lanes that share a row.
    __device__ void row_reduce() {
        for (int off = 1; off < ROW_LANES; off <<= 1) {
            cope += __shfl_xor(cope, off);
            ties += __shfl_xor(ties, off);
            borda += __shfl_xor(borda, off);
            s_out += __shfl_xor(s_out, off);
            s_in += __shfl_xor(s_in, off);
            mx_out = max(mx_out, __shfl_xor(mx_out, off));
            mx_in = max(mx_in, __shfl_xor(mx_in, off));
            mn = min(mn, __shfl_xor(mn, off));
            mx = max(mx, __shfl_xor(mx, off));
        }
    }
    // An empty asm that takes and returns every field: sums of one column
    // group are folded in here instead of being reassociated with those of
    // the next groups (which would keep every LDS value of the tile live).
    __device__ void pin() {
        asm volatile("" : "+v"(cope), "+v"(ties), "+v"(mx_out), "+v"(mx_in), "+v"(mn), "+v"(mx), "+v"(borda),
                     "+v"(s_out), "+v"(s_in));
    }
    __device__ void store(const RawStats &st, int64_t q) const {
        st.cope[q] = cope;
        st.ties[q] = ties;
        st.max_out[q] = mx_out;
        st.max_in[q] = mx_in;
        st.min_marg[q] = mn;
        st.max_marg[q] = mx;
        st.borda[q] = borda;
        st.sum_out[q] = s_out;
        st.sum_in[q] = s_in;
    }
};

// Column y of candidate x's row, xy = d[x][y], yx = d[y][x]; wo and wi are
// the edge weights x -> y and y -> x (Section 3: d[x][y] when it beats
// d[y][x], else 0, or the positive margin).
template <typename E, bool MARGIN>
__device__ __forceinline__ void acc_add(Acc<E> &s, int32_t xy, int32_t yx, int32_t &wo, int32_t &wi) {
    using S = typename Acc<E>::S;
    const int32_t marg = xy - yx;
    s.cope += xy > yx;
    s.ties += xy == yx;
    s.borda += (S)(uint32_t)xy;
    s.mn = min(s.mn, marg);
    s.mx = max(s.mx, marg);
    if (MARGIN) {
        wo = max(marg, 0);
        wi = max(-marg, 0);
    } else {
        wo = xy > yx ? xy : 0;
        wi = yx > xy ? yx : 0;
    }
    s.mx_out = max(s.mx_out, wo);
    s.mx_in = max(s.mx_in, wi);
    s.s_out += (S)(uint32_t)wo;
    s.s_in += (S)(uint32_t)wi;
}

// One lane's share of a tile: row r of the rows starting at row0 over the
// columns starting at col0, with A[r][c] = d[row0 + r][col0 + c] and
// B[c][r] = d[col0 + c][row0 + r].  The lane takes columns
// c = 8V k + V g + u (V elements per 16-byte vector).  Interior tiles of
// aligned matrices, off the diagonal.
template <typename E, bool MARGIN>
__device__ __forceinline__ void tile_rows(const E (*A)[tio::PITCH], const E (*B)[tio::PITCH], int r, int g,
                                          Acc<E> &s) {
    constexpr int V = 16 / (int)sizeof(E), KV = tio::T / (ROW_LANES * V);
    for (int k = 0; k < KV; ++k) {
        for (int u = 0; u < V; ++u) {
            const int c = k * ROW_LANES * V + g * V + u;
            int32_t wo, wi;
            acc_add<E, MARGIN>(s, (int32_t)A[r][c], (int32_t)B[c][r], wo, wi);
        }
        s.pin();
    }
}

// The same for tiles at the matrix edge, on the diagonal or of unaligned
// matrices: bounds and the diagonal checked, one element at a time (a
// plain loop: these tiles are few, and unrolling them would cost the
// interior loop registers).
template <typename E, bool MARGIN>
__device__ __forceinline__ void tile_rows_edge(const E (*A)[tio::PITCH], const E (*B)[tio::PITCH], int r, int g,
                                               int32_t row0, int32_t col0, int32_t m, Acc<E> &s) {
    constexpr int V = 16 / (int)sizeof(E);
    const int32_t x = row0 + r;
    if (x >= m) return;
#pragma unroll 1
    for (int q = 0; q < tio::T / ROW_LANES; ++q) {
        const int c = (q / V) * ROW_LANES * V + g * V + q % V, y = col0 + c;
        if (y >= m || y == x) continue;
        int32_t wo, wi;
        acc_add<E, MARGIN>(s, (int32_t)A[r][c], (int32_t)B[c][r], wo, wi);
    }
}

// Partial statistics over pairs of super-blocks (SBV x SBV tiles of 64),
// reading every block of d once.  The workgroup of super-block pair
// (I, J), I <= J, walks the tile pairs (X, Y) of I x J (of I x I only those
// with X <= Y), X outer, and loads d[X][Y] and d[Y][X] into LDS: the rows
// of X gain the columns of Y (registers rs, stored when X is done) and,
// X != Y, the rows of Y gain the columns of X (reduced over the eight lanes
// of a row and added to mir[j], in LDS, per tile of J; stored at the end).
// Slot s of each partial array holds a candidate's statistics over the
// columns of super-block s: rows of I over J and rows of J over I, each
// (row, slot) written by exactly one workgroup (on the diagonal
// super-block, row tile i adds what the tiles before it gave it as
// mirrored rows).  VD: d is read in 16-byte vectors (see tio::fetch).
template <typename E, bool MARGIN, int SBV, bool VD>
__global__ __launch_bounds__(256) void k_feature_rows(const E *__restrict__ d, int64_t ldd, int32_t m, RawStats part) {
    __shared__ E a[tio::T][tio::PITCH];  // a[r][c] = d[X0 + r][Y0 + c]
    __shared__ E b[tio::T][tio::PITCH];  // b[r][c] = d[Y0 + r][X0 + c]
    __shared__ Acc<E> mir[SBV][tio::T];
    const int32_t I = blockIdx.y, J = blockIdx.x;
    if (J < I) return;
    const int32_t nb = (m + 63) / 64;
    const int lane = threadIdx.x & 63;
    // rows r + h ROW_STEP, ROW_LANES lanes per row
    const int r = (threadIdx.x >> 6) * (64 / ROW_LANES) + lane / ROW_LANES, g = lane % ROW_LANES;
    if (g == 0)
        for (int q = 0; q < SBV; ++q) {  // read and written by this lane only
            for (int h = 0; h < RPT; ++h) mir[q][r + h * ROW_STEP].init();
        }
    // The tile pairs in order: i outer, j from i (diagonal super-block) or
    // 0; the next pair's tiles are fetched into registers while the current
    // pair is processed.
    auto valid = [&](int32_t i, int32_t j) { return i < SBV && j < SBV && I * SBV + i < nb && J * SBV + j < nb; };
    auto advance = [&](int32_t &i, int32_t &j) {  // the pair after (i, j); i = SBV when none is left
        if (valid(i, j + 1)) {
            ++j;
            return;
        }
        ++i;
        j = I == J ? i : 0;
        if (!valid(i, j)) i = SBV;
    };
    tio::Regs<E> ga, gb;
    auto fetch_pair = [&](int32_t i, int32_t j) {
        const int32_t X0 = (I * SBV + i) * 64, Y0 = (J * SBV + j) * 64;
        tio::fetch<E, VD>(ga, d, ldd, X0, Y0, m, m);
        if (X0 != Y0) tio::fetch<E, VD>(gb, d, ldd, Y0, X0, m, m);
    };
    int32_t i = 0, j = 0;
    if (!valid(i, j)) i = SBV;
    if (i < SBV) fetch_pair(i, j);
    Acc<E> rs[RPT];
    for (int h = 0; h < RPT; ++h) rs[h].init();
    while (i < SBV) {
        const int32_t X = I * SBV + i, Y = J * SBV + j;
        const int32_t X0 = X * 64, Y0 = Y * 64;
        __syncthreads();  // the previous tile pair's LDS reads are done
        tio::put<E>(a, ga);
        if (X != Y) tio::put<E>(b, gb);
        int32_t ni = i, nj = j;
        advance(ni, nj);
        if (ni < SBV) fetch_pair(ni, nj);  // in flight during the work below
        __syncthreads();
        if (X == Y) {
            for (int h = 0; h < RPT; ++h)
                tile_rows_edge<E, MARGIN>(a, a, r + h * ROW_STEP, g, X0, Y0, m, rs[h]);
        } else {
            for (int h = 0; h < RPT; ++h) {
                const int rr = r + h * ROW_STEP;
                Acc<E> ms;
                ms.init();
                if (X0 + 64 <= m && Y0 + 64 <= m) {
                    tile_rows<E, MARGIN>(a, b, rr, g, rs[h]);
                    tile_rows<E, MARGIN>(b, a, rr, g, ms);
                } else {
                    tile_rows_edge<E, MARGIN>(a, b, rr, g, X0, Y0, m, rs[h]);
                    tile_rows_edge<E, MARGIN>(b, a, rr, g, Y0, X0, m, ms);
                }
                ms.row_reduce();
                if (g == 0) mir[j][rr].merge(ms);
            }
        }
        if (ni != i) {  // the last pair of row tile X: its rows are complete over J
            for (int h = 0; h < RPT; ++h) {
                const int rr = r + h * ROW_STEP;
                rs[h].row_reduce();
                if (g == 0 && X0 + rr < m) {
                    if (I == J) rs[h].merge(mir[i][rr]);  // what the tiles before X gave its rows as mirrored rows
                    rs[h].store(part, (int64_t)J * m + X0 + rr);
                }
                rs[h].init();
            }
        }
        i = ni;
        j = nj;
    }
    if (I == J || g != 0) return;
    for (int q = 0; q < SBV; ++q)
        for (int h = 0; h < RPT; ++h) {
            const int32_t y = (J * SBV + q) * 64 + r + h * ROW_STEP;
            if (y < m) mir[q][r + h * ROW_STEP].store(part, (int64_t)I * m + y);
        }
}

// Combine the S slices' partial statistics of each candidate: a workgroup
// takes 64 candidates, its four wavefronts every fourth slice, and the four
// partial results meet in LDS (a thread per candidate alone left too few
// workgroups to keep the reads in flight).
__global__ __launch_bounds__(256) void k_feature_reduce(int32_t m, int32_t S, RawStats part, RawStats st) {
    __shared__ int32_t si[3][64][6];
    __shared__ unsigned long long su[3][64][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t x = blockIdx.x * 64 + lane;
    int32_t v[6] = {0, 0, 0, 0, INT32_MAX, INT32_MIN};  // cope, ties, max out, max in, min margin, max margin
    unsigned long long u[3] = {0, 0, 0};                // borda, sum out, sum in
    if (x < m)
        for (int32_t sl = wv; sl < S; sl += 4) {
            const int64_t q = (int64_t)sl * m + x;
            v[0] += part.cope[q];
            v[1] += part.ties[q];
            v[2] = max(v[2], part.max_out[q]);
            v[3] = max(v[3], part.max_in[q]);
            v[4] = min(v[4], part.min_marg[q]);
            v[5] = max(v[5], part.max_marg[q]);
            u[0] += part.borda[q];
            u[1] += part.sum_out[q];
            u[2] += part.sum_in[q];
        }
    if (wv > 0) {
        for (int k = 0; k < 6; ++k) si[wv - 1][lane][k] = v[k];
        for (int k = 0; k < 3; ++k) su[wv - 1][lane][k] = u[k];
    }
    __syncthreads();
    if (wv != 0 || x >= m) return;
    for (int o = 0; o < 3; ++o) {
        v[0] += si[o][lane][0];
        v[1] += si[o][lane][1];
        v[2] = max(v[2], si[o][lane][2]);
        v[3] = max(v[3], si[o][lane][3]);
        v[4] = min(v[4], si[o][lane][4]);
        v[5] = max(v[5], si[o][lane][5]);
        for (int k = 0; k < 3; ++k) u[k] += su[o][lane][k];
    }
    st.cope[x] = v[0];
    st.ties[x] = v[1];
    st.max_out[x] = v[2];
    st.max_in[x] = v[3];
    st.min_marg[x] = m > 1 ? v[4] : 0;
    st.max_marg[x] = m > 1 ? v[5] : 0;
    st.borda[x] = u[0];
    st.sum_out[x] = u[1];
    st.sum_in[x] = u[2];
}

// Maxima over candidates of the Copeland score, the largest outgoing weight
// and the Borda score: mx[0], mx[1] (int32 as uint32) and mx[2] (64 bits at
// mx + 2); zero on entry.
__global__ __launch_bounds__(256) void k_feature_max(int32_t m, RawStats st, uint32_t *__restrict__ mx) {
    __shared__ uint32_t sc, so;
    __shared__ unsigned long long sb;
    if (threadIdx.x == 0) {
        sc = 0;
        so = 0;
        sb = 0;
    }
    __syncthreads();
    const int32_t x = blockIdx.x * 256 + threadIdx.x;
    if (x < m) {
        atomicMax(&sc, (uint32_t)st.cope[x]);
        atomicMax(&so, (uint32_t)st.max_out[x]);
        atomicMax(&sb, st.borda[x]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&mx[0], sc);
        atomicMax(&mx[1], so);
        atomicMax(reinterpret_cast<unsigned long long *>(mx + 2), sb);
    }
}

// Normalise: one thread per candidate.
__global__ __launch_bounds__(256) void k_feature_norm(int32_t m, RawStats st, float n_voters,
                                                      const uint32_t *__restrict__ mx, float *__restrict__ feat) {
    const int32_t x = blockIdx.x * 256 + threadIdx.x;
    if (x >= m) return;
    const uint32_t mcope = mx[0], mout = mx[1];
    const unsigned long long mborda = *reinterpret_cast<const unsigned long long *>(mx + 2);
    const float inv_m1 = m > 1 ? 1.0f / (float)(m - 1) : 0.0f;
    const float inv_n = n_voters > 0.f ? 1.0f / n_voters : 1.0f;
    float *f = feat + (int64_t)x * NF;
    f[0] = (float)st.cope[x] * inv_m1;
    f[1] = (float)st.ties[x] * inv_m1;
    f[2] = (float)st.borda[x] * inv_m1 * inv_n;
    f[3] = (float)st.max_out[x] * inv_n;
    f[4] = (float)st.max_in[x] * inv_n;
    f[5] = st.max_in[x] > st.max_out[x] ? 1.0f : 0.0f;
    f[6] = (float)st.sum_out[x] * inv_m1 * inv_n;
    f[7] = (float)st.sum_in[x] * inv_m1 * inv_n;
    f[8] = (float)st.min_marg[x] * inv_n;
    f[9] = (float)st.max_marg[x] * inv_n;
    f[10] = logf((float)m) * 0.1f;
    f[11] = mcope > 0 ? (float)st.cope[x] / (float)mcope : 0.0f;
    f[12] = mborda > 0 ? (float)((double)st.borda[x] / (double)mborda) : 0.0f;
    f[13] = mout > 0 ? (float)st.max_out[x] / (float)mout : 0.0f;
    f[14] = ((float)st.max_out[x] - (float)st.max_in[x]) * inv_n;
    f[15] = 1.0f;
}

// Carve the nine statistic arrays of n entries each out of p.
RawStats carve(char *p, size_t n, size_t *bytes) {
    const size_t i4 = round_up(sizeof(int32_t) * n, 256), i8 = round_up(8 * n, 256);
    RawStats st;
    int32_t *const i32[6] = {reinterpret_cast<int32_t *>(p), reinterpret_cast<int32_t *>(p + i4),
                             reinterpret_cast<int32_t *>(p + 2 * i4), reinterpret_cast<int32_t *>(p + 3 * i4),
                             reinterpret_cast<int32_t *>(p + 4 * i4), reinterpret_cast<int32_t *>(p + 5 * i4)};
    st.cope = i32[0];
    st.ties = i32[1];
    st.max_out = i32[2];
    st.max_in = i32[3];
    st.min_marg = i32[4];
    st.max_marg = i32[5];
    st.borda = reinterpret_cast<unsigned long long *>(p + 6 * i4);
    st.sum_out = reinterpret_cast<unsigned long long *>(p + 6 * i4 + i8);
    st.sum_in = reinterpret_cast<unsigned long long *>(p + 6 * i4 + 2 * i8);
    *bytes = 6 * i4 + 3 * i8;
    return st;
}

template <typename E, int SBV, bool VD>
int launch_rows(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, RawStats part,
                int32_t S) {
    const dim3 grid((unsigned)S, (unsigned)S);
    if (mode == SCHULZE_MARGIN)
        SCHULZE_LAUNCH(ctx, K_FEATURE_ROWS, s,
                       k_feature_rows<E, true, SBV, VD><<<grid, dim3(256), 0, s>>>(d, ldd, m, part));
    else
        SCHULZE_LAUNCH(ctx, K_FEATURE_ROWS, s,
                       k_feature_rows<E, false, SBV, VD><<<grid, dim3(256), 0, s>>>(d, ldd, m, part));
    return SCHULZE_OK;
}

// Tiles per super-block side: more tiles mean fewer partial slots to write
// and reduce, fewer mean less LDS per workgroup (more workgroups per CU).
template <typename E>
constexpr int feature_sb() {
    return 4;
}

template <typename E>
int run_features(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, float n_voters,
                 float *feat) {
    constexpr int SBV = feature_sb<E>();
    // S super-blocks per side: a partial slot per super-block column
    const int32_t S = (int32_t)ceil_div(ceil_div(m, 64), SBV);
    size_t fin_bytes = 0, part_bytes = 0;
    (void)carve(nullptr, (size_t)m, &fin_bytes);
    (void)carve(nullptr, (size_t)m * S, &part_bytes);
    int rc = ws_reserve(ctx, WS_FEATURES, fin_bytes + part_bytes + 256);
    if (rc != SCHULZE_OK) return rc;
    char *p = static_cast<char *>(ctx->ws[WS_FEATURES]);
    RawStats st = carve(p, (size_t)m, &fin_bytes);
    RawStats part = carve(p + fin_bytes, (size_t)m * S, &part_bytes);
    uint32_t *mx = reinterpret_cast<uint32_t *>(p + fin_bytes + part_bytes);
    if ((rc = fill_u32(ctx, s, mx, 4, 0u)) != SCHULZE_OK) return rc;
    const bool vd = tio::vec_ok<E>(d, ldd) && m % (16 / (int)sizeof(E)) == 0;
    rc = vd ? launch_rows<E, SBV, true>(ctx, s, d, ldd, m, mode, part, S)
            : launch_rows<E, SBV, false>(ctx, s, d, ldd, m, mode, part, S);
    if (rc != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_FEATURES, s,
                   k_feature_reduce<<<dim3((unsigned)ceil_div(m, 64)), dim3(256), 0, s>>>(m, S, part, st));
    const dim3 vg((unsigned)ceil_div(m, 256));
    SCHULZE_LAUNCH(ctx, K_FEATURES, s, k_feature_max<<<vg, dim3(256), 0, s>>>(m, st, mx));
    SCHULZE_LAUNCH(ctx, K_FEATURES, s, k_feature_norm<<<vg, dim3(256), 0, s>>>(m, st, n_voters, mx, feat));
    return SCHULZE_OK;
}

}  // namespace

extern "C" int schulze_features(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m, int dtype,
                                int mode, float n_voters, float *feat) {
    if (!ctx || !d || !feat) return SCHULZE_EINVAL;
    if (m < 1 || ldd < m) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (m > 65535) return SCHULZE_EUNSUPPORTED;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16)
        return run_features(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode, n_voters, feat);
    return run_features(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode, n_voters, feat);
}
