// Learned proposal with exact verification.
//
// The proposer network scores every candidate from its features; the best
// candidate that the initialisation filter of Section 4 does not rule out is
// checked exactly (widest paths from and to it, the NL-membership argument
// of Section 3).  If some candidate beats it, the check moves to the
// highest-scored beater; beats is a strict partial order, so every such step
// gets closer to a winner.  Once a winner c is found, every other winner is
// tied with c (winners do not beat each other), so the winner set is c plus
// the tied candidates that pass the same check.  If no winner is found
// within max_climb steps, or too many candidates are tied, the full closure
// decides.  The output is always exactly the Schulze winner set.
#include <vector>

#include "internal.h"

namespace {

// argmax of score over candidates the filter keeps (feat[x][5] == 0);
// ties -> lowest id; out[0] = candidate or -1 if every candidate is filtered.
// One workgroup of 1024 threads, four candidates per thread in flight, a
// wavefront maximum, then one LDS atomic per wavefront.
constexpr int PROPOSE_THREADS = 1024;
__global__ __launch_bounds__(PROPOSE_THREADS) void k_propose(const float *__restrict__ score,
                                                             const float *__restrict__ feat, int32_t m,
                                                             int use_filter, int32_t *out) {
    __shared__ unsigned long long best;
    if (threadIdx.x == 0) best = 0ull;
    __syncthreads();
    unsigned long long mine = 0ull;
    for (int32_t x0 = threadIdx.x; x0 < m; x0 += 4 * PROPOSE_THREADS) {
        float sc[4], fl[4];
        for (int u = 0; u < 4; ++u) {  // loads first, so that they are in flight together
            const int32_t x = x0 + u * PROPOSE_THREADS;
            const int32_t xc = x < m ? x : 0;
            sc[u] = score[xc];
            fl[u] = use_filter ? feat[(int64_t)xc * 16 + 5] : 0.0f;
        }
        for (int u = 0; u < 4; ++u) {
            const int32_t x = x0 + u * PROPOSE_THREADS;
            if (x >= m || fl[u] != 0.0f) continue;
            const uint32_t bits = __float_as_uint(sc[u]);
            const uint32_t key = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
            const unsigned long long k = ((unsigned long long)key << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)x);
            mine = k > mine ? k : mine;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off);
        mine = o > mine ? o : mine;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(&best, mine);
    __syncthreads();
    if (threadIdx.x == 0) out[0] = best ? (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull)) : -1;
}

// The winner set of a search that found at most MAX_LISTED winners:
// is_winner[j] = 1 for the listed ids, 0 elsewhere; *n_winners = count.
constexpr int MAX_LISTED = 64;
struct WinnerList {
    int32_t n;
    int32_t id[MAX_LISTED];
};
__global__ __launch_bounds__(256) void k_set_winners(uint8_t *__restrict__ is_winner, int32_t m, WinnerList list,
                                                     int32_t *n_winners) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < m) {
        uint8_t v = 0;
        for (int k = 0; k < list.n; ++k) v |= list.id[k] == j ? 1 : 0;
        is_winner[j] = v;
    }
    if (j == 0 && n_winners) *n_winners = list.n;
}

// score[x] = feat[x][col]: the proposers that rank by one feature column.
__global__ __launch_bounds__(256) void k_score_column(const float *__restrict__ feat, int32_t m, int32_t col,
                                                      float *__restrict__ score) {
    const int32_t x = blockIdx.x * 256 + threadIdx.x;
    if (x < m) score[x] = feat[(int64_t)x * 16 + col];
}

}  // namespace

extern "C" int schulze_set_proposer(schulze_ctx *ctx, int proposer) {
    if (!ctx || proposer < SCHULZE_PROPOSER_NETWORK || proposer > SCHULZE_PROPOSER_FILTER_BORDA) return SCHULZE_EINVAL;
    ctx->proposer = proposer;
    return SCHULZE_OK;
}

extern "C" int schulze_winners_learned(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                                       int dtype, int mode, float n_voters, const float *params, int32_t max_climb,
                                       int32_t max_tied, uint8_t *is_winner, int32_t *n_winners,
                                       schulze_learned_stats *stats) {
    if (!ctx || !d || !is_winner) return SCHULZE_EINVAL;
    const int proposer = ctx->proposer;
    if (proposer == SCHULZE_PROPOSER_NETWORK && !params) return SCHULZE_EINVAL;
    if (m < 1 || ldd < m || max_climb < 0 || max_tied < 0) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (m > 65535) return SCHULZE_EUNSUPPORTED;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const size_t es = dtype == SCHULZE_U16 ? 2 : 4;
    const size_t mat = round_up(es * (size_t)m * m, 256);
    const size_t vec_e = round_up(es * (size_t)m, 256), vec_f = round_up(4 * (size_t)m, 256);
    const size_t feat_b = round_up(4 * 16 * (size_t)m, 256);
    int rc = ws_reserve(ctx, WS_LEARNED, feat_b + vec_f + 2 * vec_e + vec_f + 256);
    if (rc != SCHULZE_OK) return rc;
    char *b = static_cast<char *>(ctx->ws[WS_LEARNED]);
    float *feat = reinterpret_cast<float *>(b);
    float *score = reinterpret_cast<float *>(b + feat_b);
    void *p_from = b + feat_b + vec_f;
    void *p_to = b + feat_b + vec_f + vec_e;
    int32_t *tied = reinterpret_cast<int32_t *>(b + feat_b + vec_f + 2 * vec_e);
    int32_t *small = reinterpret_cast<int32_t *>(b + feat_b + 2 * vec_f + 2 * vec_e);  // verdict + pick

    schulze_learned_stats st{};
    st.proposal = -1;
    // features in one pass over d (nothing else written)
    if ((rc = schulze_features(ctx, stream, d, ldd, m, dtype, mode, n_voters, feat)) != SCHULZE_OK) return rc;
    // scores: the network, or one feature column (Borda: column 2, the vertex
    // order of Section 4; Copeland: column 0); the filter of Section 4 applies
    // to the network and to filtered Borda
    if (proposer == SCHULZE_PROPOSER_NETWORK) {
        if ((rc = schulze_mlp_forward(ctx, stream, params, feat, m, score)) != SCHULZE_OK) return rc;
    } else {
        const int32_t col = proposer == SCHULZE_PROPOSER_COPELAND ? 0 : 2;
        SCHULZE_LAUNCH(ctx, K_PROPOSE, s,
                       k_score_column<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s>>>(feat, m, col, score));
    }
    const int use_filter = proposer == SCHULZE_PROPOSER_NETWORK || proposer == SCHULZE_PROPOSER_FILTER_BORDA;
    SCHULZE_LAUNCH(ctx, K_PROPOSE, s,
                   k_propose<<<dim3(1), dim3(PROPOSE_THREADS), 0, s>>>(score, feat, m, use_filter, small + 4));
    int32_t cand = -1;
    if (hipMemcpyAsync(&cand, small + 4, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SCHULZE_EDEVICE;
    if (cand < 0) {  // every candidate filtered: cannot happen for consistent data; score all
        SCHULZE_LAUNCH(ctx, K_PROPOSE, s, k_propose<<<dim3(1), dim3(PROPOSE_THREADS), 0, s>>>(score, feat, m, 0, small + 4));
        if (hipMemcpyAsync(&cand, small + 4, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SCHULZE_EDEVICE;
    }
    st.proposal = cand;

    // One exact check.  The first reads d itself (schulze_verify_counts:
    // weights formed where they are used, nothing written first), which
    // suits the common case of a proposal that wins outright.  A search that
    // goes on (a climb, tied candidates) writes the weights once, then
    // sweeps over their rows: int32 counts as the signed weights w - w^T
    // (both directions read rows of one matrix), 16-bit counts as w and w^T.
    // The verdict is only used when the device error word is clear: a
    // widest-path launch that gave up on its bounded grid barrier leaves its
    // rows unwritten and sets the word, so the search stops with
    // SCHULZE_EDEVICE (the word stays set for schulze_get_device_error)
    // instead of deciding on stale rows.
    void *w = nullptr, *wt = nullptr;
    const bool sgn = dtype == SCHULZE_I32;
    auto verify = [&](int32_t c, int32_t (&v)[4]) -> int {
        int r;
        if (st.verify_calls == 0) {
            r = schulze_verify_counts(ctx, stream, d, ldd, m, dtype, mode, c, score, p_from, p_to, small, tied);
        } else {
            if (!w) {
                if ((r = ws_reserve(ctx, WS_LEARNED_W, (sgn ? 1 : 2) * mat)) != SCHULZE_OK) return r;
                char *wb = static_cast<char *>(ctx->ws[WS_LEARNED_W]);
                if (sgn) {
                    r = signed_weights(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode,
                                       reinterpret_cast<int32_t *>(wb), m);
                } else {
                    r = schulze_weights(ctx, stream, d, ldd, m, dtype, mode, wb, m, wb + mat, m);
                }
                if (r != SCHULZE_OK) return r;
                w = wb;
                wt = sgn ? nullptr : wb + mat;
            }
            r = sgn ? verify_signed(ctx, s, static_cast<const int32_t *>(w), m, m, c, score,
                                    static_cast<int32_t *>(p_from), static_cast<int32_t *>(p_to), small, tied)
                    : schulze_verify(ctx, stream, w, m, wt, m, m, dtype, c, score, p_from, p_to, small, tied);
        }
        if (r != SCHULZE_OK) return r;
        ++st.verify_calls;
        int32_t err = 0;
        if (hipMemcpyAsync(v, small, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&err, ctx->err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SCHULZE_EDEVICE;
        return err == SCHULZE_OK ? SCHULZE_OK : SCHULZE_EDEVICE;
    };

    int32_t v[4];
    int32_t winner = -1;
    for (int32_t step = 0; step <= max_climb; ++step) {
        if ((rc = verify(cand, v)) != SCHULZE_OK) return rc;
        if (step == 0) st.first_hit = v[0];
        if (v[0]) {
            winner = cand;
            break;
        }
        if (step == max_climb || v[2] < 0) break;
        cand = v[2];
        ++st.climbs;
    }
    std::vector<uint8_t> host_win;
    if (winner >= 0 && v[3] <= max_tied) {
        std::vector<int32_t> ties(v[3]);
        if (v[3] > 0 &&
            (hipMemcpyAsync(ties.data(), tied, sizeof(int32_t) * v[3], hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            return SCHULZE_EDEVICE;
        host_win.assign(m, 0);
        host_win[winner] = 1;
        for (int32_t t : ties) {
            int32_t vt[4];
            if ((rc = verify(t, vt)) != SCHULZE_OK) return rc;
            if (vt[0]) host_win[t] = 1;
        }
        int32_t nw = 0;
        for (uint8_t x : host_win) nw += x;
        st.n_winners = nw;
        if (nw <= MAX_LISTED) {  // the usual case: the few ids as kernel arguments, no host-to-device copy
            WinnerList list{};
            for (int32_t x = 0; x < m; ++x)
                if (host_win[x]) list.id[list.n++] = x;
            // (asynchronous: the ids travel as kernel arguments)
            SCHULZE_LAUNCH(ctx, K_WINNERS, s,
                           k_set_winners<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s>>>(is_winner, m, list,
                                                                                               n_winners));
        } else {
            if (hipMemcpyAsync(is_winner, host_win.data(), (size_t)m, hipMemcpyHostToDevice, s) != hipSuccess)
                return SCHULZE_EDEVICE;
            if (n_winners && hipMemcpyAsync(n_winners, &st.n_winners, sizeof(int32_t), hipMemcpyHostToDevice, s) !=
                                 hipSuccess)
                return SCHULZE_EDEVICE;
            if (hipStreamSynchronize(s) != hipSuccess) return SCHULZE_EDEVICE;  // host buffers end with this call
        }
    } else {
        // fallback: the full closure decides
        st.fallback = 1;
        if ((rc = ws_reserve(ctx, WS_LEARNED_P, mat)) != SCHULZE_OK) return rc;
        void *p = ctx->ws[WS_LEARNED_P];
        if ((rc = schulze_closure(ctx, stream, d, ldd, m, dtype, mode, p, m)) != SCHULZE_OK) return rc;
        if ((rc = schulze_winners(ctx, stream, p, m, m, dtype, is_winner, n_winners ? n_winners : small + 8)) !=
            SCHULZE_OK)
            return rc;
        int32_t nw = 0;
        if (hipMemcpyAsync(&nw, n_winners ? n_winners : small + 8, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SCHULZE_EDEVICE;
        st.n_winners = nw;
    }
    if (stats) *stats = st;
    return SCHULZE_OK;
}
