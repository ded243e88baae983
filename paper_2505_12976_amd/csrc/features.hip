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

struct RawStats {
    int32_t *cope, *ties;
    unsigned long long *borda, *sum_out, *sum_in;
    int32_t *max_out, *max_in;
    long long *min_marg, *max_marg;
};

// Statistics of one candidate over a set of columns.
struct Stat {
    int32_t cope, ties, mx_out, mx_in;
    unsigned long long borda, s_out, s_in;
    long long mn, mxm;
};

__device__ inline void stat_init(Stat &s) {
    s.cope = s.ties = s.mx_out = s.mx_in = 0;
    s.borda = s.s_out = s.s_in = 0ull;
    s.mn = LLONG_MAX;
    s.mxm = LLONG_MIN;
}

// One column y of candidate x's row: dxy = d[x][y], dyx = d[y][x].
__device__ inline void stat_add(Stat &s, int64_t dxy, int64_t dyx, int mode) {
    s.cope += dxy > dyx;
    s.ties += dxy == dyx;
    s.borda += (unsigned long long)dxy;
    const long long marg = dxy - dyx;
    s.mn = min(s.mn, marg);
    s.mxm = max(s.mxm, marg);
    const int32_t wout = dxy > dyx ? (int32_t)(mode == SCHULZE_MARGIN ? dxy - dyx : dxy) : 0;
    const int32_t win = dyx > dxy ? (int32_t)(mode == SCHULZE_MARGIN ? dyx - dxy : dyx) : 0;
    s.mx_out = max(s.mx_out, wout);
    s.mx_in = max(s.mx_in, win);
    s.s_out += (unsigned long long)wout;
    s.s_in += (unsigned long long)win;
}

__device__ inline void stat_merge(Stat &s, const Stat &o) {
    s.cope += o.cope;
    s.ties += o.ties;
    s.borda += o.borda;
    s.s_out += o.s_out;
    s.s_in += o.s_in;
    s.mx_out = max(s.mx_out, o.mx_out);
    s.mx_in = max(s.mx_in, o.mx_in);
    s.mn = min(s.mn, o.mn);
    s.mxm = max(s.mxm, o.mxm);
}

// Combine the statistics of the 4 adjacent lanes that share a row.
__device__ inline void stat_quad_reduce(Stat &s) {
    for (int off = 1; off < 4; off <<= 1) {
        s.cope += __shfl_xor(s.cope, off);
        s.ties += __shfl_xor(s.ties, off);
        s.borda += __shfl_xor(s.borda, off);
        s.s_out += __shfl_xor(s.s_out, off);
        s.s_in += __shfl_xor(s.s_in, off);
        s.mx_out = max(s.mx_out, __shfl_xor(s.mx_out, off));
        s.mx_in = max(s.mx_in, __shfl_xor(s.mx_in, off));
        s.mn = min(s.mn, (long long)__shfl_xor(s.mn, off));
        s.mxm = max(s.mxm, (long long)__shfl_xor(s.mxm, off));
    }
}

__device__ inline void stat_store(const RawStats &st, int64_t q, const Stat &s) {
    st.cope[q] = s.cope;
    st.ties[q] = s.ties;
    st.borda[q] = s.borda;
    st.sum_out[q] = s.s_out;
    st.sum_in[q] = s.s_in;
    st.max_out[q] = s.mx_out;
    st.max_in[q] = s.mx_in;
    st.min_marg[q] = s.mn;
    st.max_marg[q] = s.mxm;
}

constexpr int SB_MAX = 8;  // 64-tiles per side of a super-block

// Partial statistics over pairs of super-blocks, reading every block of d
// once.  The matrix is cut into super-blocks of sb x sb tiles of 64; the
// workgroup of super-block pair (I, J), I <= J, walks the tile pairs
// (X, Y) in I x J (in I x I only those with X <= Y) and loads d[X][Y] and
// d[Y][X] together: rows of X gain the columns of Y (kept in registers over
// the tiles of J) and, X != Y, rows of Y gain the columns of X (kept in LDS
// per tile of J, over the tiles of I).  Slot s of each partial array holds a
// candidate's statistics over the columns of super-block s: rows of I over
// J and rows of J over I, each (row, slot) written by exactly one
// workgroup.  With w / wt given, the same pass writes the edge weights of
// both tiles of each pair to w and to its transpose wt.
template <typename E>
__global__ __launch_bounds__(256) void k_feature_rows(const E *__restrict__ d, int64_t ldd, int32_t m, int mode,
                                                      RawStats part, int vec, E *__restrict__ w, int64_t ldw,
                                                      E *__restrict__ wt, int64_t ldwt, int32_t sb) {
    __shared__ E a[64][65];  // a[r][c] = d[X0 + r][Y0 + c]
    __shared__ E b[64][65];  // b[r][c] = d[Y0 + r][X0 + c]
    __shared__ Stat mir[SB_MAX][64];
    const int32_t I = blockIdx.y, J = blockIdx.x;
    if (J < I) return;
    const int32_t nb = (m + 63) / 64;
    const int r = threadIdx.x >> 2, part_c = threadIdx.x & 3;  // 4 threads per row, 16 columns each
    if (part_c == 0)
        for (int j = 0; j < SB_MAX; ++j) stat_init(mir[j][r]);
    auto weight = [&](E xy, E yx, bool diag) -> E {  // edge weight given d[i][j] = xy, d[j][i] = yx
        if (diag || xy <= yx) return (E)0;
        return mode == SCHULZE_MARGIN ? (E)(xy - yx) : xy;
    };
    for (int32_t i = 0; i < sb; ++i) {
        const int32_t X = I * sb + i;
        if (X >= nb) break;
        const int32_t X0 = X * 64, x = X0 + r;
        Stat rs;
        stat_init(rs);
        for (int32_t j = I == J ? i : 0; j < sb; ++j) {
            const int32_t Y = J * sb + j;
            if (Y >= nb) break;
            const int32_t Y0 = Y * 64;
            __syncthreads();
            tio::load<E>(a, d, ldd, X0, Y0, m, m, (vec & 1) != 0);
            if (X != Y) tio::load<E>(b, d, ldd, Y0, X0, m, m, (vec & 1) != 0);
            __syncthreads();
            const E(*bb)[65] = X != Y ? b : a;  // d[Y0 + r][X0 + c]
            if (w) {
                tio::store<E>(w, ldw, X0, Y0, m, m, (vec & 2) != 0,
                              [&](int rr, int cc) { return weight(a[rr][cc], bb[cc][rr], X0 + rr == Y0 + cc); });
                if (X != Y)
                    tio::store<E>(w, ldw, Y0, X0, m, m, (vec & 2) != 0,
                                  [&](int rr, int cc) { return weight(bb[rr][cc], a[cc][rr], false); });
            }
            if (wt) {
                tio::store<E>(wt, ldwt, Y0, X0, m, m, (vec & 4) != 0,
                              [&](int rr, int cc) { return weight(a[cc][rr], bb[rr][cc], X0 + cc == Y0 + rr); });
                if (X != Y)
                    tio::store<E>(wt, ldwt, X0, Y0, m, m, (vec & 4) != 0,
                                  [&](int rr, int cc) { return weight(bb[cc][rr], a[rr][cc], false); });
            }
            // rows of X over the columns of Y
            if (x < m)
                for (int c = part_c * 16; c < part_c * 16 + 16; ++c) {
                    const int32_t y = Y0 + c;
                    if (y < m && y != x) stat_add(rs, a[r][c], bb[c][r], mode);
                }
            if (X != Y) {  // rows of Y over the columns of X
                Stat ms;
                stat_init(ms);
                const int32_t yr = Y0 + r;
                if (yr < m)
                    for (int c = part_c * 16; c < part_c * 16 + 16; ++c)
                        if (X0 + c < m) stat_add(ms, bb[r][c], a[c][r], mode);
                stat_quad_reduce(ms);
                if (part_c == 0) stat_merge(mir[j][r], ms);  // only this thread touches mir[j][r]
            }
        }
        stat_quad_reduce(rs);
        if (part_c == 0 && x < m) {
            // on the diagonal super-block, tile X's rows also hold the columns of
            // the tiles before it (gathered as mirrored rows)
            if (I == J) stat_merge(rs, mir[i][r]);
            stat_store(part, (int64_t)J * m + x, rs);
        }
    }
    if (I == J) return;
    for (int32_t j = 0; j < sb; ++j) {
        const int32_t Y = J * sb + j;
        if (Y >= nb) break;
        const int32_t y = Y * 64 + r;
        if (part_c == 0 && y < m) stat_store(part, (int64_t)I * m + y, mir[j][r]);
    }
}

// Combine the S slices' partial statistics of each candidate.
__global__ __launch_bounds__(256) void k_feature_reduce(int32_t m, int32_t S, RawStats part, RawStats st) {
    const int32_t x = blockIdx.x * 256 + threadIdx.x;
    if (x >= m) return;
    int32_t cope = 0, ties = 0, mx_out = 0, mx_in = 0;
    unsigned long long borda = 0, s_out = 0, s_in = 0;
    long long mn = LLONG_MAX, mxm = LLONG_MIN;
    for (int32_t sl = 0; sl < S; ++sl) {
        const int64_t q = (int64_t)sl * m + x;
        cope += part.cope[q];
        ties += part.ties[q];
        borda += part.borda[q];
        s_out += part.sum_out[q];
        s_in += part.sum_in[q];
        mx_out = max(mx_out, part.max_out[q]);
        mx_in = max(mx_in, part.max_in[q]);
        mn = min(mn, part.min_marg[q]);
        mxm = max(mxm, part.max_marg[q]);
    }
    st.cope[x] = cope;
    st.ties[x] = ties;
    st.borda[x] = borda;
    st.sum_out[x] = s_out;
    st.sum_in[x] = s_in;
    st.max_out[x] = mx_out;
    st.max_in[x] = mx_in;
    st.min_marg[x] = m > 1 ? mn : 0;
    st.max_marg[x] = m > 1 ? mxm : 0;
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
    st.cope = reinterpret_cast<int32_t *>(p);
    st.ties = reinterpret_cast<int32_t *>(p + i4);
    st.max_out = reinterpret_cast<int32_t *>(p + 2 * i4);
    st.max_in = reinterpret_cast<int32_t *>(p + 3 * i4);
    st.borda = reinterpret_cast<unsigned long long *>(p + 4 * i4);
    st.sum_out = reinterpret_cast<unsigned long long *>(p + 4 * i4 + i8);
    st.sum_in = reinterpret_cast<unsigned long long *>(p + 4 * i4 + 2 * i8);
    st.min_marg = reinterpret_cast<long long *>(p + 4 * i4 + 3 * i8);
    st.max_marg = reinterpret_cast<long long *>(p + 4 * i4 + 4 * i8);
    *bytes = 4 * i4 + 5 * i8;
    return st;
}

template <typename E>
int run_features(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, float n_voters,
                 float *feat, E *w = nullptr, int64_t ldw = 0, E *wt = nullptr, int64_t ldwt = 0) {
    // super-blocks of sb x sb tiles: at most 64 of them per side (a partial
    // slot per super-block column), sb <= SB_MAX; S = super-blocks per side
    const int32_t nbx = (int32_t)ceil_div(m, 64);
    int32_t sb = 1;
    while (sb < SB_MAX && ceil_div(nbx, sb) > 64) sb *= 2;
    const int32_t S = (int32_t)ceil_div(nbx, sb);
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
    const int vec = (tio::vec_ok<E>(d, ldd) ? 1 : 0) | (tio::vec_ok<E>(w, ldw) ? 2 : 0) |
                    (tio::vec_ok<E>(wt, ldwt) ? 4 : 0);
    SCHULZE_LAUNCH(ctx, K_FEATURE_ROWS, s,
                   k_feature_rows<E><<<dim3((unsigned)S, (unsigned)S), dim3(256), 0, s>>>(
                       d, ldd, m, mode, part, vec, w, ldw, wt, ldwt, sb));
    SCHULZE_LAUNCH(ctx, K_FEATURES, s,
                   k_feature_reduce<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s>>>(m, S, part, st));
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

// Internal: features and both weight matrices in one pass over d (the
// learned path needs all three).
int weights_and_features(schulze_ctx *ctx, hipStream_t s, const void *d, int64_t ldd, int32_t m, int dtype, int mode,
                         float n_voters, float *feat, void *w, int64_t ldw, void *wt, int64_t ldwt) {
    if (dtype == SCHULZE_U16)
        return run_features(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode, n_voters, feat,
                            static_cast<uint16_t *>(w), ldw, static_cast<uint16_t *>(wt), ldwt);
    return run_features(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode, n_voters, feat,
                        static_cast<int32_t *>(w), ldw, static_cast<int32_t *>(wt), ldwt);
}
