// Edge weights and single-source / single-target widest paths.
//
// Winner verification follows the NL-membership argument of Section 3: a
// candidate c is a Schulze winner iff for every other candidate x the widest
// c->x path is at least as wide as the widest x->c path.  Both families of
// widths are computed exactly with (max, min) relaxation sweeps:
//     x_s[j] <- max(x_s[j], max_i min(x_s[i], w[i][j])),
// started from x_s[s] = MAX and 0 elsewhere.  The values only grow, each is
// the width of some path, and after k sweeps every path of <= k edges has
// been seen, so the fixpoint is the widest-path row p[s][.] (at most m - 1
// sweeps).  Only rows whose value grew in the previous sweep can raise
// anything, so each sweep walks just that frontier.  The target direction
// p[.][t] is the same computation on the transposed weights.
//
// One persistent cooperative launch runs all sweeps (the column-block and
// frontier-share layout of sweep.h), with a grid barrier between sweeps.
#include <mutex>

#include "grid.h"
#include "sweep.h"
#include "tile_io.h"

// Device scratch of schulze_verify_noalloc: the sweeps' value vector, flags,
// two frontier lists and counters for up to 65535 candidates (852 KB used
// at that size).  Each device holds its own copy for the life of the
// process.  In host code `scratch` only names the symbol; its device address
// comes from hipGetSymbolAddress (verify_scratch_init) and is the only form
// passed to kernels.
constexpr size_t VERIFY_SCRATCH_BYTES = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[VERIFY_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};  // device address of `scratch`, per device

}  // namespace

// Look up this device's address of the scratch array (once per device; the
// device must be current).
int verify_scratch_init(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return SCHULZE_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SCHULZE_EDEVICE;
        }
        g_scratch[device] = p;
    }
    *ptr = g_scratch[device];
    return SCHULZE_OK;
}

namespace {

using grid::GridBar;
using grid::grid_sync;

template <typename E>
__device__ inline E max_value() {
    return sizeof(E) == 2 ? (E)0xFFFF : (E)0x7FFFFFFF;
}

// ------------------------------------------------------------------ weights
// w[i][j] and wt[j][i] = edge weight of (i, j) from d (winning votes or
// margin).  A workgroup takes the 64 x 64 blocks (I, J) and (J, I), I <= J,
// of both outputs: they need the same two blocks of d, read once.
template <typename E>
__global__ __launch_bounds__(256) void k_weights_pair(const E *__restrict__ d, int64_t ldd, int32_t m, int mode,
                                                      E *__restrict__ w, int64_t ldw, E *__restrict__ wt,
                                                      int64_t ldwt, int vec) {
    __shared__ E a[64][65];  // a[r][c] = d[I0 + r][J0 + c]
    __shared__ E b[64][65];  // b[r][c] = d[J0 + r][I0 + c]
    if (blockIdx.y > blockIdx.x) return;
    const int32_t I0 = blockIdx.y * 64, J0 = blockIdx.x * 64;
    tio::load<E>(a, d, ldd, I0, J0, m, m, vec & 1);
    tio::load<E>(b, d, ldd, J0, I0, m, m, vec & 1);
    __syncthreads();
    auto weight = [&](E x, E y, bool diag) -> E {  // weight of edge (i, j) given d[i][j] = x, d[j][i] = y
        if (diag || x <= y) return (E)0;
        return mode == SCHULZE_MARGIN ? (E)(x - y) : x;
    };
    const bool wv = (vec & 2) != 0, wtv = (vec & 4) != 0;
    // edges (I0 + r, J0 + c) into w; edges (I0 + c, J0 + r) into wt row J0 + r
    if (w) tio::store<E>(w, ldw, I0, J0, m, m, wv, [&](int r, int c) { return weight(a[r][c], b[c][r], I0 + r == J0 + c); });
    if (wt) tio::store<E>(wt, ldwt, J0, I0, m, m, wtv, [&](int r, int c) { return weight(a[c][r], b[r][c], I0 + c == J0 + r); });
    if (I0 == J0) return;
    // edges (J0 + r, I0 + c) into w; edges (J0 + c, I0 + r) into wt row I0 + r
    if (w) tio::store<E>(w, ldw, J0, I0, m, m, wv, [&](int r, int c) { return weight(b[r][c], a[c][r], false); });
    if (wt) tio::store<E>(wt, ldwt, I0, J0, m, m, wtv, [&](int r, int c) { return weight(b[c][r], a[r][c], false); });
}

// ------------------------------------------------------------------ grid barrier
// ------------------------------------------------------------------ sweeps
template <typename E>
struct WidestArgs {
    const E *w;          // rows = sources of edges (w, or wt for the target direction)
    int64_t ldw;
    int32_t m;
    int32_t s;           // source (or target) vertex
    int32_t vec;         // rows of w allow 8/16-byte accesses
    E *out;              // m widths, out[s] = 0
    uint32_t *x;         // m values, in place
    uint8_t *changed;    // m flags
    int32_t *front[2];   // frontier lists (m entries each)
    int32_t *fcount;     // [0], [1]: frontier sizes; [2]: sweeps run
    GridBar *bar;
    int32_t *err;
    int64_t spin_limit;
};

template <typename E>
__global__ __launch_bounds__(256) void k_widest(WidestArgs<E> a) {
    const int32_t m = a.m;
    // x = MAX at s, 0 elsewhere; frontier = {s}
    for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) {
        a.x[j] = j == a.s ? (uint32_t)max_value<E>() : 0u;
        a.changed[j] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.front[0][0] = a.s;
        a.fcount[0] = 1;
        a.fcount[1] = 0;
    }
    if (!grid_sync(a.bar, a.spin_limit)) goto stuck;
    {
        sweep::Buffers<uint32_t> b{a.x, {a.front[0], a.front[1]}, a.fcount, a.changed, a.bar, a.err, a.spin_limit,
                                   m + 1};
        const bool ok = sweep::run<uint32_t, E>(
            a.w, a.ldw, m, a.vec != 0, b, [](uint32_t xi, uint32_t e) { return min(xi, e); },
            [](int32_t) { return true; });
        if (!ok) goto stuck;
        for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256)
            a.out[j] = j == a.s ? (E)0 : (E)a.x[j];
        return;
    }
stuck:
    if (threadIdx.x == 0) set_device_error(a.err, SCHULZE_EDEVICE);
}

// ------------------------------------------------------------------ verdict
// out[0] = 1 if c is a winner; out[1] = number of candidates beating c;
// out[2] = a beater (highest score, or widest margin p(x,c) - p(c,x) when
// no scores are given; ties -> lowest id) or -1; out[3] = number of x != c
// tied with c (p(c,x) = p(x,c)).  tied[] (optional) lists them.
template <typename E>
__global__ __launch_bounds__(256) void k_verdict(const E *__restrict__ from, const E *__restrict__ to, int32_t m,
                                                 int32_t c, const float *__restrict__ score, int32_t *out,
                                                 int32_t *tied) {
    __shared__ int32_t nbeat, ntie;
    __shared__ unsigned long long best;
    if (threadIdx.x == 0) {
        nbeat = 0;
        ntie = 0;
        best = 0ull;
    }
    __syncthreads();
    for (int32_t x = threadIdx.x; x < m; x += 256) {
        if (x == c) continue;
        const E f = from[x], t = to[x];
        if (t > f) {
            atomicAdd(&nbeat, 1);
            // key: larger is better; ids ascending on ties
            uint32_t hi;
            if (score) {
                const float sc = score[x];
                uint32_t bits = __float_as_uint(sc);
                hi = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);  // order-preserving
            } else {
                hi = (uint32_t)(t - f);
            }
            const unsigned long long key = ((unsigned long long)hi << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)x);
            atomicMax(&best, key);
        } else if (t == f) {
            const int32_t k = atomicAdd(&ntie, 1);
            if (tied) tied[k] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = nbeat == 0 ? 1 : 0;
        out[1] = nbeat;
        out[2] = nbeat ? (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull)) : -1;
        out[3] = ntie;
    }
}

// 8-byte (uint16) or 16-byte (int32) row accesses of a matrix at p, pitch ld.
template <typename E>
bool sweep_vec_ok(const void *p, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(p) % (4 * sizeof(E)) == 0) && (ld % 4 == 0);
}

// Scratch of one widest-path launch: values, flags, two frontiers, counters, barrier.
size_t widest_scratch_bytes(int32_t m) {
    const size_t xbytes = round_up(sizeof(uint32_t) * (size_t)m, 256);
    const size_t cbytes = round_up((size_t)m, 256);
    const size_t fbytes = round_up(sizeof(int32_t) * (size_t)m, 256);
    return xbytes + cbytes + 2 * fbytes + 256;
}

// Widest paths from src over the rows of w, with the sweep state in `base`
// (widest_scratch_bytes(m) bytes of device memory; the counters and barrier
// are cleared here, everything else is written before it is read).  `timed`
// brackets the launch with the context's timing events.
template <typename E>
int widest_in(schulze_ctx *ctx, hipStream_t s, const E *w, int64_t ldw, int32_t m, int32_t src, E *out, char *base,
              bool timed) {
    const size_t xbytes = round_up(sizeof(uint32_t) * (size_t)m, 256);
    const size_t cbytes = round_up((size_t)m, 256);
    const size_t fbytes = round_up(sizeof(int32_t) * (size_t)m, 256);
    int rc;
    WidestArgs<E> a;
    a.w = w;
    a.ldw = ldw;
    a.m = m;
    a.s = src;
    a.vec = sweep_vec_ok<E>(w, ldw) ? 1 : 0;
    a.out = out;
    a.x = reinterpret_cast<uint32_t *>(base);
    a.changed = reinterpret_cast<uint8_t *>(base + xbytes);
    a.front[0] = reinterpret_cast<int32_t *>(base + xbytes + cbytes);
    a.front[1] = reinterpret_cast<int32_t *>(base + xbytes + cbytes + fbytes);
    int32_t *tail = reinterpret_cast<int32_t *>(base + xbytes + cbytes + 2 * fbytes);
    a.fcount = tail;
    a.bar = reinterpret_cast<GridBar *>(tail + 8);
    a.err = ctx->err;
    a.spin_limit = (int64_t)1 << 24;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(tail), 64, 0u)) != SCHULZE_OK) return rc;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_widest<E>, 256, 0) != hipSuccess || per_cu < 1)
        return SCHULZE_EDEVICE;
    const int64_t G = sweep::grid_size(m, (int64_t)ctx->num_cus * std::min(per_cu, 2));
    void *args[] = {&a};
    int tok = -1;
    if (timed) timing_begin(ctx, K_WIDEST, s, &tok);
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_widest<E>, dim3((unsigned)G), dim3(256), args, 0, s);
    if (timed) timing_end(ctx, tok, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SCHULZE_EDEVICE;
    }
    return SCHULZE_OK;
}

template <typename E>
int widest(schulze_ctx *ctx, hipStream_t s, const E *w, int64_t ldw, int32_t m, int32_t src, E *out) {
    int rc = ws_reserve(ctx, WS_VERIFY, widest_scratch_bytes(m));
    if (rc != SCHULZE_OK) return rc;
    return widest_in<E>(ctx, s, w, ldw, m, src, out, static_cast<char *>(ctx->ws[WS_VERIFY]), true);
}

// Both widest-path directions and the verdict, with the sweep state in base
// (nullptr: the context's workspace).
template <typename E>
int verify_all(schulze_ctx *ctx, hipStream_t s, const E *w, int64_t ldw, const E *wt, int64_t ldwt, int32_t m,
               int32_t cand, const float *score, E *p_from, E *p_to, int32_t *verdict, int32_t *tied, char *base) {
    int rc;
    if (base) {
        if ((rc = widest_in<E>(ctx, s, w, ldw, m, cand, p_from, base, false)) != SCHULZE_OK) return rc;
        if ((rc = widest_in<E>(ctx, s, wt, ldwt, m, cand, p_to, base, false)) != SCHULZE_OK) return rc;
        k_verdict<E><<<dim3(1), dim3(256), 0, s>>>(p_from, p_to, m, cand, score, verdict, tied);
        return launch_status();
    }
    if ((rc = widest<E>(ctx, s, w, ldw, m, cand, p_from)) != SCHULZE_OK) return rc;
    if ((rc = widest<E>(ctx, s, wt, ldwt, m, cand, p_to)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_VERDICT, s,
                   k_verdict<E><<<dim3(1), dim3(256), 0, s>>>(p_from, p_to, m, cand, score, verdict, tied));
    return SCHULZE_OK;
}

int check_square(schulze_ctx *ctx, const void *a, int64_t ld, int32_t m, int dtype) {
    if (!ctx || !a) return SCHULZE_EINVAL;
    if (m < 1 || ld < m) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (m > 65535) return SCHULZE_EUNSUPPORTED;
    return bind_device(ctx);
}

}  // namespace

extern "C" int schulze_weights(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m, int dtype,
                               int mode, void *w, int64_t ldw, void *wt, int64_t ldwt) {
    int rc = check_square(ctx, d, ldd, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (!w && !wt) return SCHULZE_EINVAL;
    if ((w && ldw < m) || (wt && ldwt < m)) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(m, 64));
    if (dtype == SCHULZE_U16) {
        const int vec = (tio::vec_ok<uint16_t>(d, ldd) ? 1 : 0) | (tio::vec_ok<uint16_t>(w, ldw) ? 2 : 0) |
                        (tio::vec_ok<uint16_t>(wt, ldwt) ? 4 : 0);
        SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                       k_weights_pair<uint16_t><<<grid, dim3(256), 0, s>>>(
                           static_cast<const uint16_t *>(d), ldd, m, mode, static_cast<uint16_t *>(w), ldw,
                           static_cast<uint16_t *>(wt), ldwt, vec));
    } else {
        const int vec = (tio::vec_ok<int32_t>(d, ldd) ? 1 : 0) | (tio::vec_ok<int32_t>(w, ldw) ? 2 : 0) |
                        (tio::vec_ok<int32_t>(wt, ldwt) ? 4 : 0);
        SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                       k_weights_pair<int32_t><<<grid, dim3(256), 0, s>>>(
                           static_cast<const int32_t *>(d), ldd, m, mode, static_cast<int32_t *>(w), ldw,
                           static_cast<int32_t *>(wt), ldwt, vec));
    }
    return SCHULZE_OK;
}

extern "C" int schulze_widest_from(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, int32_t m, int dtype,
                                   int32_t source, void *out) {
    int rc = check_square(ctx, w, ldw, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (!out || source < 0 || source >= m) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16)
        return widest<uint16_t>(ctx, s, static_cast<const uint16_t *>(w), ldw, m, source, static_cast<uint16_t *>(out));
    return widest<int32_t>(ctx, s, static_cast<const int32_t *>(w), ldw, m, source, static_cast<int32_t *>(out));
}

extern "C" int schulze_verify(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, const void *wt,
                              int64_t ldwt, int32_t m, int dtype, int32_t cand, const float *score, void *p_from,
                              void *p_to, int32_t *verdict, int32_t *tied) {
    int rc = check_square(ctx, w, ldw, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (!wt || ldwt < m || !p_from || !p_to || !verdict || cand < 0 || cand >= m) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16) {
        using E = uint16_t;
        return verify_all<E>(ctx, s, static_cast<const E *>(w), ldw, static_cast<const E *>(wt), ldwt, m, cand, score,
                             static_cast<E *>(p_from), static_cast<E *>(p_to), verdict, tied, nullptr);
    }
    using E = int32_t;
    return verify_all<E>(ctx, s, static_cast<const E *>(w), ldw, static_cast<const E *>(wt), ldwt, m, cand, score,
                         static_cast<E *>(p_from), static_cast<E *>(p_to), verdict, tied, nullptr);
}

extern "C" int schulze_verify_noalloc(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, const void *wt,
                                      int64_t ldwt, int32_t m, int dtype, int32_t cand, const float *score,
                                      void *p_from, void *p_to, int32_t *verdict, int32_t *tied) {
    int rc = check_square(ctx, w, ldw, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (!wt || ldwt < m || !p_from || !p_to || !verdict || cand < 0 || cand >= m) return SCHULZE_EINVAL;
    if (widest_scratch_bytes(m) > VERIFY_SCRATCH_BYTES) return SCHULZE_EUNSUPPORTED;
    if (!ctx->verify_scratch) return SCHULZE_EDEVICE;  // set when the context was created
    char *base = static_cast<char *>(ctx->verify_scratch);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16) {
        using E = uint16_t;
        return verify_all<E>(ctx, s, static_cast<const E *>(w), ldw, static_cast<const E *>(wt), ldwt, m, cand, score,
                             static_cast<E *>(p_from), static_cast<E *>(p_to), verdict, tied, base);
    }
    using E = int32_t;
    return verify_all<E>(ctx, s, static_cast<const E *>(w), ldw, static_cast<const E *>(wt), ldwt, m, cand, score,
                         static_cast<E *>(p_from), static_cast<E *>(p_to), verdict, tied, base);
}
