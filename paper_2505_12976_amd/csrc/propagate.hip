// Schulze winners by forward/backward propagation of minimum labels with
// path widths: the paper's own winners-only algorithm (Section 4: the
// initialisation filter, then rounds of preprocessing, forward-backward
// propagation and postprocessing until no candidate is undecided), run as
// dense data-parallel sweeps over the weight matrix instead of Pregel
// messages.
//
// Labels.  Every undecided candidate carries a label, its position in the
// chosen vertex order (Borda scores descending, ties by id, as Section 4
// suggests; or plain ids).  Forward, each vertex keeps the smallest label
// that reaches it with the width of the widest path from that candidate;
// backward, the smallest label it reaches with the widest path width to it.
// Decided candidates carry no label but pass labels on.  A label and a width
// are packed into one key -- (LABEL_MAX - label) in the high half, the width
// in the low half -- so "smaller label, then wider path" is a plain max of
// keys, and along an edge of weight w > 0 a key k becomes
// (k & HIGH) | min(k & LOW, w).  Sweeps run to the fixpoint; only vertices
// whose key grew in a sweep send in the next one.  At the fixpoint, for a
// vertex with label s, every vertex on a path from s has label s as well, so
// its width is the widest-path width p(s, c).
//
// Postprocessing of a vertex c with forward (s, ws) and backward (t, wt):
//   s < t   c is reached from s but does not reach it: s beats c;
//   s > t   c reaches t and t does not reach c: c beats t;
//   s = t   c and s share a strongly connected component (the vertices with
//           (s, t) = (x, x) are exactly x's component); ws > wt: s beats c,
//           ws < wt: c beats s;
//   an edge v -> c whose (s, t) differ from c's crosses components (vertices
//   of one component share (s, t)), so c does not reach v and v beats c,
//   and every vertex of c's component when s = t.
// After all marks of a round, an undecided c whose own label is s = t (the
// smallest undecided vertex of its component) and that is still undecided
// has no beater: nobody outside its component reaches it and nobody inside
// beats it.  It wins.  Every round decides at least the smallest undecided
// label, so there are at most m rounds.
#include "grid.h"
#include "sweep.h"

namespace {

using grid::GridBar;
using grid::grid_sync;

// ST_REMOVED: taken out of the election (top-k: a winner of an earlier
// round); such a vertex has no edges, so it neither holds nor relays labels.
enum : uint8_t { ST_UNKNOWN = 0, ST_LOSER = 1, ST_WINNER = 2, ST_REMOVED = 3 };

template <typename E>
struct Key;
template <>
struct Key<uint16_t> {
    using K = uint32_t;
    static constexpr int SH = 16;
    static constexpr uint32_t WMAX = 0xFFFFu;    // width of the empty path
    static constexpr uint32_t LMAX = 0xFFFFu;    // labels are < LMAX
    static constexpr K LOW = 0xFFFFu;
};
template <>
struct Key<int32_t> {
    using K = unsigned long long;
    static constexpr int SH = 32;
    static constexpr uint32_t WMAX = 0x7FFFFFFFu;
    static constexpr uint32_t LMAX = 0xFFFFFFFFu;
    static constexpr K LOW = 0xFFFFFFFFull;
};

template <typename E>
__device__ inline typename Key<E>::K make_key(uint32_t label) {
    using KT = Key<E>;
    return ((typename KT::K)(KT::LMAX - label) << KT::SH) | (typename KT::K)KT::WMAX;
}

// label of a key, or 0xFFFFFFFF for none
template <typename E>
__device__ inline uint32_t key_label(typename Key<E>::K k) {
    using KT = Key<E>;
    const uint32_t code = (uint32_t)(k >> KT::SH);
    return code == 0 ? 0xFFFFFFFFu : KT::LMAX - code;
}

template <typename E>
__device__ inline uint32_t key_width(typename Key<E>::K k) {
    return (uint32_t)(k & Key<E>::LOW);
}

// Four consecutive elements of a row starting at a multiple of 4 (one 8- or
// 16-byte access when vec and all four are inside, else one at a time, 0
// past `valid`).
template <typename E>
__device__ inline void load4(const E *__restrict__ p, bool vec, int32_t valid, uint32_t (&v)[4]) {
    if (vec && valid >= 4) {
        if constexpr (sizeof(E) == 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(p);
            v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
        } else {
            const uint2 q = *reinterpret_cast<const uint2 *>(p);
            v[0] = q.x & 0xFFFFu, v[1] = q.x >> 16, v[2] = q.y & 0xFFFFu, v[3] = q.y >> 16;
        }
    } else {
        for (int c = 0; c < 4; ++c) v[c] = c < valid ? (uint32_t)p[c] : 0u;
    }
}

// ------------------------------------------------------------------ per-vertex statistics
// Row x of w and of wt among the vertices still in (rem[y] = 0): largest
// outgoing and incoming edge weight (the initialisation filter) and, when
// with_borda, the Borda score sum_y d[x][y].  Every vertex still in starts
// undecided unless the filter rules it out; removed vertices get ST_REMOVED.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_rows(const E *__restrict__ d, int64_t ldd, const E *__restrict__ w,
                                                   const E *__restrict__ wt, int64_t ld, int32_t m,
                                                   const uint8_t *__restrict__ rem, int with_borda, int vec,
                                                   uint8_t *__restrict__ status, unsigned long long *__restrict__ borda) {
    __shared__ uint32_t smax_out[256], smax_in[256];
    __shared__ unsigned long long sb[256];
    const int32_t x = blockIdx.x;
    if (rem[x]) {
        if (threadIdx.x == 0) status[x] = ST_REMOVED;
        return;
    }
    // int32: w holds the signed weights S = w - w^T and wt is unused
    constexpr bool SGN = sizeof(E) == 4;
    uint32_t mo = 0, mi = 0;
    unsigned long long b = 0;
    const E *wr = w + (int64_t)x * ld, *wtr = SGN ? wr : wt + (int64_t)x * ld, *dr = d + (int64_t)x * ldd;
    // four columns per thread and step: 8- or 16-byte accesses where the rows allow them
    const bool wv = (vec & 1) != 0, dv = (vec & 2) != 0;
    for (int32_t y0 = threadIdx.x * 4; y0 < m; y0 += 1024) {
        uint32_t a[4], at[4], ad[4] = {0u, 0u, 0u, 0u};
        uint8_t r[4];
        const bool full = y0 + 4 <= m;
        if (full && wv) {
            load4<E>(wr + y0, true, 4, a);
            if (!SGN) load4<E>(wtr + y0, true, 4, at);
            const uint32_t rw = *reinterpret_cast<const uint32_t *>(rem + y0);
            for (int u = 0; u < 4; ++u) r[u] = (uint8_t)(rw >> (8 * u));
        } else {
            for (int u = 0; u < 4; ++u) {
                const bool in = y0 + u < m;
                a[u] = in ? (uint32_t)wr[y0 + u] : 0u;
                if (!SGN) at[u] = in ? (uint32_t)wtr[y0 + u] : 0u;
                r[u] = in ? rem[y0 + u] : (uint8_t)1;
            }
        }
        if constexpr (SGN)
            for (int u = 0; u < 4; ++u) {
                const int32_t v = (int32_t)a[u];
                a[u] = (uint32_t)max(v, 0);
                at[u] = (uint32_t)max(-v, 0);
            }
        if (with_borda) load4<E>(dr + y0, full && dv, full ? 4 : m - y0, ad);
        for (int u = 0; u < 4; ++u) {
            if (r[u]) continue;
            mo = max(mo, a[u]);
            mi = max(mi, at[u]);
            if (y0 + u != x) b += (unsigned long long)ad[u];
        }
    }
    smax_out[threadIdx.x] = mo;
    smax_in[threadIdx.x] = mi;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smax_out[threadIdx.x] = max(smax_out[threadIdx.x], smax_out[threadIdx.x + off]);
            smax_in[threadIdx.x] = max(smax_in[threadIdx.x], smax_in[threadIdx.x + off]);
            sb[threadIdx.x] += sb[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        status[x] = smax_in[0] > smax_out[0] ? ST_LOSER : ST_UNKNOWN;  // initialisation filter
        if (with_borda) borda[x] = sb[0];
    }
}

// label[x] = position of x in the order (Borda descending, then id), or x;
// vertex[label] = x.
__global__ __launch_bounds__(256) void k_prop_order(const unsigned long long *__restrict__ borda, int32_t m,
                                                    int use_borda, int32_t *__restrict__ label,
                                                    int32_t *__restrict__ vertex) {
    __shared__ int32_t part[256];
    const int32_t x = blockIdx.x;
    int32_t r = 0;
    if (use_borda) {
        const unsigned long long bx = borda[x];
        for (int32_t y = threadIdx.x; y < m; y += 256) {
            const unsigned long long by = borda[y];
            r += (by > bx || (by == bx && y < x)) ? 1 : 0;
        }
    }
    part[threadIdx.x] = r;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int32_t lx = use_borda ? part[0] : x;
        label[x] = lx;
        vertex[lx] = x;
    }
}

// ------------------------------------------------------------------ propagation sweeps
// Both directions in one launch: problem 0 propagates forward over the
// rows of w into kf, problem 1 backward over the rows of wt into kb (int32:
// both over the rows of the signed weights S, as max(S, 0) and max(-S, 0)).
template <typename E>
struct SweepArgs {
    sweep::Run<typename Key<E>::K, E, 2> run;
    int32_t m;
    const uint8_t *status;
    const int32_t *label;
};

// Undecided vertices start with their own label and the empty path; they
// form the first frontier of both directions.  The counters and the barrier
// are zero on entry.  A plain launch ahead of the sweeps.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_init(SweepArgs<E> a) {
    using K = typename Key<E>::K;
    const int32_t m = a.m;
    const int lane = threadIdx.x & 63;
    for (int32_t j0 = blockIdx.x * 256; j0 < m; j0 += gridDim.x * 256) {
        const int32_t j = j0 + threadIdx.x;
        const bool u = j < m && a.status[j] == ST_UNKNOWN;
        const uint64_t bal = __ballot(u);
        for (int q = 0; q < 2; ++q) {
            const sweep::Problem<K, E> &P = a.run.p[q];
            if (j < m) {
                P.x[j] = u ? make_key<E>((uint32_t)a.label[j]) : (K)0;
                P.stamp[j] = 0;
            }
            int32_t base = 0;
            if (lane == 0 && bal) base = atomicAdd(&P.count[0], (int32_t)__popcll(bal));
            base = __shfl(base, 0);
            if (u) P.front[0][base + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = j;
        }
    }
}

template <typename E>
__global__ __launch_bounds__(256) void k_prop_sweep(SweepArgs<E> a) {
    using K = typename Key<E>::K;
    constexpr K HIGH = ~Key<E>::LOW;
    const uint8_t *status = a.status;
    const bool ok = sweep::run<K, E, 2>(
        a.run, a.m,
        [](int q, K k, uint32_t wij) -> K {
            if constexpr (sizeof(E) == 4) {  // signed weights: problem 0 takes max(S, 0), problem 1 max(-S, 0)
                const int32_t v = q ? -(int32_t)wij : (int32_t)wij;
                wij = (uint32_t)max(v, 0);
            }
            if (wij == 0 || k == 0) return (K)0;
            return (k & HIGH) | (K)min((uint32_t)(k & Key<E>::LOW), wij);
        },
        [status](int32_t j) { return status[j] != ST_REMOVED; });  // removed vertices have no edges
    if (!ok && threadIdx.x == 0) set_device_error(a.run.err, SCHULZE_EDEVICE);
}

// ------------------------------------------------------------------ postprocessing
// Marks from each vertex's own (s, ws, t, wt).  mark[v] = 1: v is beaten;
// dead[x] = 1: the component labelled x is beaten.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_post(const typename Key<E>::K *__restrict__ kf,
                                                   const typename Key<E>::K *__restrict__ kb, int32_t m,
                                                   const int32_t *__restrict__ vertex, uint8_t *__restrict__ mark) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= m) return;
    const uint32_t s = key_label<E>(kf[c]), t = key_label<E>(kb[c]);
    if (s == 0xFFFFFFFFu && t == 0xFFFFFFFFu) return;  // joined to no undecided vertex
    if (s < t) {
        mark[c] = 1;
    } else if (s > t) {
        mark[vertex[t]] = 1;
    } else {
        const uint32_t ws = key_width<E>(kf[c]), wt = key_width<E>(kb[c]);
        if (ws > wt)
            mark[c] = 1;
        else if (ws < wt)
            mark[vertex[s]] = 1;
    }
}

// Each vertex's (s, t) in one word: labels are below 65534, "no label" is
// PAIR_NONE, and a removed vertex (no edges) gets PAIR_OUT in both halves.
constexpr uint32_t PAIR_NONE = 0xFFFEu;
constexpr uint32_t PAIR_OUT = 0xFFFFFFFFu;

template <typename E>
__global__ __launch_bounds__(256) void k_prop_pair(const typename Key<E>::K *__restrict__ kf,
                                                   const typename Key<E>::K *__restrict__ kb, int32_t m,
                                                   const uint8_t *__restrict__ status, uint32_t *__restrict__ pair) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= m) return;
    const uint32_t s = key_label<E>(kf[v]), t = key_label<E>(kb[v]);
    pair[v] = status[v] == ST_REMOVED ? PAIR_OUT
                                       : ((s == 0xFFFFFFFFu ? PAIR_NONE : s) << 16) | (t == 0xFFFFFFFFu ? PAIR_NONE : t);
}

// Edges v -> c between vertices with different (s, t): one wavefront per c
// walks column c of w (row c of wt), four entries per lane and step.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_cross(const E *__restrict__ wt, int64_t ld,
                                                    const uint32_t *__restrict__ pair, int32_t m, int vec,
                                                    uint8_t *__restrict__ mark, uint8_t *__restrict__ dead) {
    const int32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= m) return;
    const uint32_t pc = pair[c];
    if (pc == PAIR_OUT) return;
    const E *row = wt + (int64_t)c * ld;
    bool cross = false;
    for (int32_t v0 = lane * 4; v0 < m; v0 += 256) {
        uint32_t e[4], pv[4];
        if (vec && v0 + 4 <= m) {
            if constexpr (sizeof(E) == 4) {
                const uint4 q = *reinterpret_cast<const uint4 *>(row + v0);
                e[0] = q.x, e[1] = q.y, e[2] = q.z, e[3] = q.w;
            } else {
                const uint2 q = *reinterpret_cast<const uint2 *>(row + v0);
                e[0] = q.x & 0xFFFFu, e[1] = q.x >> 16, e[2] = q.y & 0xFFFFu, e[3] = q.y >> 16;
            }
            const uint4 p4 = *reinterpret_cast<const uint4 *>(pair + v0);
            pv[0] = p4.x, pv[1] = p4.y, pv[2] = p4.z, pv[3] = p4.w;
        } else {
            for (int u = 0; u < 4; ++u) {
                e[u] = v0 + u < m ? (uint32_t)row[v0 + u] : 0u;
                pv[u] = v0 + u < m ? pair[v0 + u] : PAIR_OUT;
            }
        }
        // an edge v -> c: wt[c][v] > 0, or with signed weights (int32) S[c][v] < 0
        for (int u = 0; u < 4; ++u)
            cross |= (sizeof(E) == 4 ? (int32_t)e[u] < 0 : e[u] != 0) && pv[u] != PAIR_OUT && pv[u] != pc;
    }
    if (__ballot(cross) && lane == 0) {
        const uint32_t s = pc >> 16, t = pc & 0xFFFFu;
        if (s == t) {
            if (s != PAIR_NONE) dead[s] = 1;
        } else {
            mark[c] = 1;
        }
    }
}

// Apply the marks to undecided vertices; then count the undecided ones.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_apply(const typename Key<E>::K *__restrict__ kf,
                                                    const typename Key<E>::K *__restrict__ kb, int32_t m,
                                                    const uint8_t *__restrict__ mark, const uint8_t *__restrict__ dead,
                                                    uint8_t *__restrict__ status) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= m || status[c] != ST_UNKNOWN) return;
    const uint32_t s = key_label<E>(kf[c]), t = key_label<E>(kb[c]);
    if (mark[c] || (s == t && s != 0xFFFFFFFFu && dead[s])) status[c] = ST_LOSER;
}

// Winners: undecided vertices whose own label is their (s, t).  counts[0]
// receives the number still undecided after this round.
template <typename E>
__global__ __launch_bounds__(256) void k_prop_decide(const typename Key<E>::K *__restrict__ kf,
                                                     const typename Key<E>::K *__restrict__ kb, int32_t m,
                                                     const int32_t *__restrict__ label, uint8_t *__restrict__ status,
                                                     int32_t *__restrict__ counts) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    int32_t undecided = 0;
    if (c < m && status[c] == ST_UNKNOWN) {
        const uint32_t s = key_label<E>(kf[c]), t = key_label<E>(kb[c]);
        if (s == (uint32_t)label[c] && t == s)
            status[c] = ST_WINNER;
        else
            undecided = 1;
    }
    const uint64_t bal = __ballot(undecided);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&counts[0], (int32_t)__popcll(bal));
}

__global__ __launch_bounds__(256) void k_prop_out(const uint8_t *__restrict__ status, int32_t m,
                                                  uint8_t *__restrict__ is_winner, int32_t *__restrict__ counts) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    int32_t win = 0;
    if (c < m) {
        win = status[c] == ST_WINNER ? 1 : 0;
        is_winner[c] = (uint8_t)win;
    }
    const uint64_t bal = __ballot(win);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&counts[1], (int32_t)__popcll(bal));
}

// Top-k: the winners of this round leave the election (level = round);
// everyone else still in becomes undecided again.  counts[0] += winners,
// counts[1] += vertices still in.
__global__ __launch_bounds__(256) void k_prop_remove(uint8_t *__restrict__ status, int32_t m, int32_t round,
                                                     int32_t *__restrict__ level, uint8_t *__restrict__ rem,
                                                     int32_t *__restrict__ counts) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    int32_t win = 0, in = 0;
    if (c < m) {
        const uint8_t st = status[c];
        if (st == ST_WINNER) {
            level[c] = round;
            rem[c] = 1;
            win = 1;
        } else if (st != ST_REMOVED) {
            in = 1;
        }
    }
    const uint64_t bw = __ballot(win), bi = __ballot(in);
    if ((threadIdx.x & 63) == 0) {
        if (bw) atomicAdd(&counts[0], (int32_t)__popcll(bw));
        if (bi) atomicAdd(&counts[1], (int32_t)__popcll(bi));
    }
}

// Access widths for k_prop_rows: bit 0 = rows of w and w^T (pitch m, in the
// workspace), bit 1 = rows of d.
template <typename E>
int rows_vec(const E *d, int64_t ldd, int32_t m) {
    const bool wv = m % 4 == 0;
    const bool dv = reinterpret_cast<uintptr_t>(d) % (4 * sizeof(E)) == 0 && ldd % 4 == 0;
    return (wv ? 1 : 0) | (dv ? 2 : 0);
}

// Device buffers of one propagation run (slices of the WS_PROPAGATE slot).
template <typename E>
struct PropBufs {
    using K = typename Key<E>::K;
    E *w, *wt;
    K *kf, *kb;
    int32_t *front[4], *stamp[2], *label, *vertex;
    uint32_t *pair;
    unsigned long long *borda;
    uint8_t *status, *mark, *dead, *rem;
    int32_t *cnt;   // sweep counters of the two directions, 64 words apart
    GridBar *bar;
    int32_t *tail;  // [16..17] counts
    size_t bvec;
    int64_t G;      // sweep grid
};

// Weights, the removal mask cleared, the filter, the Borda scores and the labels.
template <typename E>
int prop_prepare(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, int use_borda,
                 PropBufs<E> &b) {
    using K = typename Key<E>::K;
    const size_t mat = round_up(sizeof(E) * (size_t)m * m, 256);
    const size_t kvec = round_up(sizeof(K) * (size_t)m, 256);
    const size_t ivec = round_up(sizeof(int32_t) * (size_t)m, 256);
    const size_t bvec = round_up((size_t)m, 256);
    const size_t u64vec = round_up(sizeof(unsigned long long) * (size_t)m, 256);
    // w | wt | kf | kb | fronts x4 | stamps x2 | label | vertex | pair | borda | status | mark | dead | rem |
    // counters | barrier | tail
    const size_t barb = round_up(grid::BAR_BYTES, 256);
    // int32 counts keep one matrix of signed weights S = w - w^T (both weight
    // rules give a pair an edge in at most one direction): w = max(S, 0),
    // w^T = max(-S, 0); 16-bit counts keep w and w^T
    constexpr bool SGN = sizeof(E) == 4;
    const size_t need = (SGN ? 1 : 2) * mat + 2 * kvec + 9 * ivec + u64vec + 4 * bvec + 512 + barb + 256;
    int rc = ws_reserve(ctx, WS_PROPAGATE, need);
    if (rc != SCHULZE_OK) return rc;
    char *p = static_cast<char *>(ctx->ws[WS_PROPAGATE]);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += bytes;
        return q;
    };
    b.w = reinterpret_cast<E *>(take(mat));
    b.wt = SGN ? nullptr : reinterpret_cast<E *>(take(mat));
    b.kf = reinterpret_cast<K *>(take(kvec));
    b.kb = reinterpret_cast<K *>(take(kvec));
    for (int i = 0; i < 4; ++i) b.front[i] = reinterpret_cast<int32_t *>(take(ivec));
    for (int i = 0; i < 2; ++i) b.stamp[i] = reinterpret_cast<int32_t *>(take(ivec));
    b.label = reinterpret_cast<int32_t *>(take(ivec));
    b.vertex = reinterpret_cast<int32_t *>(take(ivec));
    b.pair = reinterpret_cast<uint32_t *>(take(ivec));
    b.borda = reinterpret_cast<unsigned long long *>(take(u64vec));
    b.status = reinterpret_cast<uint8_t *>(take(bvec));
    b.mark = reinterpret_cast<uint8_t *>(take(bvec));
    b.dead = reinterpret_cast<uint8_t *>(take(bvec));
    b.rem = reinterpret_cast<uint8_t *>(take(bvec));
    b.cnt = reinterpret_cast<int32_t *>(take(512));
    b.bar = reinterpret_cast<GridBar *>(take(barb));
    b.tail = reinterpret_cast<int32_t *>(take(256));
    b.bvec = bvec;

    const int dtype = sizeof(E) == 2 ? SCHULZE_U16 : SCHULZE_I32;
    if constexpr (SGN)
        rc = signed_weights(ctx, s, reinterpret_cast<const int32_t *>(d), ldd, m, mode,
                            reinterpret_cast<int32_t *>(b.w), m);
    else
        rc = schulze_weights(ctx, s, d, ldd, m, dtype, mode, b.w, m, b.wt, m);
    if (rc != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.rem), bvec / 4, 0u)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_PROP, s,
                   k_prop_rows<E><<<dim3((unsigned)m), dim3(256), 0, s>>>(d, ldd, b.w, b.wt, m, m, b.rem, 1,
                                                                         rows_vec<E>(d, ldd, m), b.status, b.borda));
    SCHULZE_LAUNCH(ctx, K_PROP, s,
                   k_prop_order<<<dim3((unsigned)m), dim3(256), 0, s>>>(b.borda, m, use_borda, b.label, b.vertex));

    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_prop_sweep<E>, 256, 0) != hipSuccess || per_cu < 1)
        return SCHULZE_EDEVICE;
    b.G = sweep::grid_size(m, 2, (int64_t)ctx->num_cus * std::min(per_cu, 2));
    return SCHULZE_OK;
}

// Rounds of forward/backward propagation, postprocessing and decisions
// until no vertex still in is undecided.
template <typename E>
int prop_decide_all(schulze_ctx *ctx, hipStream_t s, int32_t m, PropBufs<E> &b, schulze_propagate_stats &st) {
    using K = typename Key<E>::K;
    int rc;
    const unsigned vb = (unsigned)ceil_div(m, 256);
    int32_t counts[2] = {0, 0};
    for (int32_t round = 0; round < m; ++round) {
        {
            // counters and barrier cleared (adjacent), then the init and both directions' sweeps
            const size_t words = (512 + round_up(grid::BAR_BYTES, 256)) / 4;
            if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.cnt), words, 0u)) != SCHULZE_OK) return rc;
            SweepArgs<E> a;
            for (int q = 0; q < 2; ++q) {
                sweep::Problem<K, E> &P = a.run.p[q];
                P.A = (q == 0 || sizeof(E) == 4) ? b.w : b.wt;  // int32: both read the signed weights
                P.ld = m;
                P.vec = sweep::vec_ok<E>(P.A, m) ? 1 : 0;
                P.x = q == 0 ? b.kf : b.kb;
                P.stamp = b.stamp[q];
                P.front[0] = b.front[2 * q];
                P.front[1] = b.front[2 * q + 1];
                P.count = b.cnt + 64 * q;
            }
            a.run.max_sweeps = ctx->sweep_max_sweeps > 0 ? ctx->sweep_max_sweeps : 2 * m + 2;
            a.run.bar = b.bar;
            a.run.err = ctx->err;
            a.run.spin_limit = ctx->sweep_spin_limit > 0 ? ctx->sweep_spin_limit : SWEEP_SPIN_LIMIT;
            a.m = m;
            a.status = b.status;
            a.label = b.label;
            int tok;
            timing_begin(ctx, K_PROP_SWEEP, s, &tok);
            k_prop_init<E><<<dim3((unsigned)std::min<int64_t>(vb, 1024)), dim3(256), 0, s>>>(a);
            hipError_t e = hipGetLastError();
            void *args[] = {&a};
            if (e == hipSuccess)
                e = hipLaunchCooperativeKernel((const void *)k_prop_sweep<E>, dim3((unsigned)b.G), dim3(256), args, 0,
                                               s);
            timing_end(ctx, tok, s);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return SCHULZE_EDEVICE;
            }
            int32_t sweeps[2] = {0, 0}, err = 0;
            if (hipMemcpyAsync(&sweeps[0], b.cnt + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&sweeps[1], b.cnt + 64 + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&err, ctx->err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return SCHULZE_EDEVICE;
            // a sweep that gave up (the word stays set for schulze_get_device_error)
            // leaves no labels to decide on
            if (err != SCHULZE_OK) return SCHULZE_EDEVICE;
            st.sweeps += sweeps[0] + sweeps[1];
        }
        // mark and dead are adjacent: clear both
        if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.mark), 2 * b.bvec / 4, 0u)) != SCHULZE_OK) return rc;
        if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.tail + 16), 2, 0u)) != SCHULZE_OK) return rc;
        SCHULZE_LAUNCH(ctx, K_PROP, s, k_prop_post<E><<<dim3(vb), dim3(256), 0, s>>>(b.kf, b.kb, m, b.vertex, b.mark));
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_pair<E><<<dim3(vb), dim3(256), 0, s>>>(b.kf, b.kb, m, b.status, b.pair));
        const E *wtc = sizeof(E) == 4 ? b.w : b.wt;  // rows of w^T, or of the signed weights
        const int cvec = (reinterpret_cast<uintptr_t>(wtc) % (4 * sizeof(E)) == 0 && m % 4 == 0) ? 1 : 0;
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_cross<E><<<dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, s>>>(wtc, m, b.pair, m, cvec,
                                                                                            b.mark, b.dead));
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_apply<E><<<dim3(vb), dim3(256), 0, s>>>(b.kf, b.kb, m, b.mark, b.dead, b.status));
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_decide<E><<<dim3(vb), dim3(256), 0, s>>>(b.kf, b.kb, m, b.label, b.status, b.tail + 16));
        if (hipMemcpyAsync(counts, b.tail + 16, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SCHULZE_EDEVICE;
        ++st.rounds;
        if (counts[0] == 0) return SCHULZE_OK;
    }
    return SCHULZE_EDEVICE;  // more rounds than candidates: cannot happen
}

template <typename E>
int run_propagate(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, int use_borda,
                  uint8_t *is_winner, int32_t *n_winners, schulze_propagate_stats *stats) {
    PropBufs<E> b;
    int rc = prop_prepare<E>(ctx, s, d, ldd, m, mode, use_borda, b);
    if (rc != SCHULZE_OK) return rc;
    schulze_propagate_stats st{};
    if ((rc = prop_decide_all<E>(ctx, s, m, b, st)) != SCHULZE_OK) return rc;
    const unsigned vb = (unsigned)ceil_div(m, 256);
    int32_t counts[2] = {0, 0};
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.tail + 16), 2, 0u)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_PROP, s, k_prop_out<<<dim3(vb), dim3(256), 0, s>>>(b.status, m, is_winner, b.tail + 16));
    if (hipMemcpyAsync(counts, b.tail + 16, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SCHULZE_EDEVICE;
    st.n_winners = counts[1];
    if (n_winners &&
        (hipMemcpyAsync(n_winners, &st.n_winners, sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        return SCHULZE_EDEVICE;
    if (stats) *stats = st;
    return SCHULZE_OK;
}

// Top-k: winners of the candidates still in, removed, again, until at least
// k candidates have a level or none is left.
template <typename E>
int run_topk(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, int use_borda, int32_t k,
             int32_t *level, schulze_topk_stats *stats) {
    PropBufs<E> b;
    int rc = prop_prepare<E>(ctx, s, d, ldd, m, mode, use_borda, b);
    if (rc != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(level), (size_t)m, 0xFFFFFFFFu)) != SCHULZE_OK) return rc;
    const unsigned vb = (unsigned)ceil_div(m, 256);
    schulze_topk_stats out{};
    schulze_propagate_stats st{};
    for (int32_t lv = 0;; ++lv) {
        if ((rc = prop_decide_all<E>(ctx, s, m, b, st)) != SCHULZE_OK) return rc;
        if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(b.tail + 16), 2, 0u)) != SCHULZE_OK) return rc;
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_remove<<<dim3(vb), dim3(256), 0, s>>>(b.status, m, lv, level, b.rem, b.tail + 16));
        int32_t counts[2] = {0, 0};
        if (hipMemcpyAsync(counts, b.tail + 16, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SCHULZE_EDEVICE;
        if (counts[0] < 1) return SCHULZE_EDEVICE;  // every nonempty election has a winner
        out.levels = lv + 1;
        out.ranked += counts[0];
        if (out.ranked >= k || counts[1] == 0) break;
        SCHULZE_LAUNCH(ctx, K_PROP, s,
                       k_prop_rows<E><<<dim3((unsigned)m), dim3(256), 0, s>>>(d, ldd, b.w, b.wt, m, m, b.rem, 0,
                                                                             rows_vec<E>(d, ldd, m), b.status,
                                                                             b.borda));
    }
    out.rounds = st.rounds;
    out.sweeps = st.sweeps;
    if (stats) *stats = out;
    return SCHULZE_OK;
}

}  // namespace

extern "C" int schulze_winners_propagate(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                                         int dtype, int mode, int borda_order, uint8_t *is_winner,
                                         int32_t *n_winners, schulze_propagate_stats *stats) {
    if (!ctx || !d || !is_winner) return SCHULZE_EINVAL;
    if (m < 1 || ldd < m) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (m > 65534) return SCHULZE_EUNSUPPORTED;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16)
        return run_propagate<uint16_t>(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode, borda_order != 0,
                                       is_winner, n_winners, stats);
    return run_propagate<int32_t>(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode, borda_order != 0, is_winner,
                                  n_winners, stats);
}

extern "C" int schulze_topk_propagate(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                                      int dtype, int mode, int borda_order, int32_t k, int32_t *level,
                                      schulze_topk_stats *stats) {
    if (!ctx || !d || !level) return SCHULZE_EINVAL;
    if (m < 1 || ldd < m || k < 1) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (m > 65534) return SCHULZE_EUNSUPPORTED;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16)
        return run_topk<uint16_t>(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode, borda_order != 0, k, level,
                                  stats);
    return run_topk<int32_t>(ctx, s, static_cast<const int32_t *>(d), ldd, m, mode, borda_order != 0, k, level, stats);
}
