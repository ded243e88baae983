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
// Both weight rules give an edge at most one direction per pair (winning
// votes: the larger count; margin: the positive difference), so the signed
// matrix S = w - w^T holds both: w[i][j] = max(S[i][j], 0) and
// w^T[i][j] = max(-S[i][j], 0).  With int32 counts the learned path keeps
// only S, and its two directions read rows of the same matrix.
//
// One persistent cooperative launch runs all sweeps of both directions (the
// column-block and frontier-share layout of sweep.h), with one grid barrier
// per sweep.
#include <mutex>

#include "grid.h"
#include "sweep.h"
#include "tile_io.h"

// Device scratch of schulze_verify_noalloc: for both directions the sweeps'
// values, stamps, two frontier lists and counters, then the barrier, for up
// to 65535 candidates (2.1 MB used at that size).  Each device holds its own
// copy for the life of the process.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress
// (verify_scratch_init) and is the only form passed to kernels.
constexpr size_t VERIFY_SCRATCH_BYTES = (size_t)3 << 20;
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
// SIGNED (int32): w receives the signed weights w - w^T and wt is null.
template <typename E, bool SIGNED = false>
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
    if constexpr (SIGNED) {
        tio::store<E>(w, ldw, I0, J0, m, m, wv, [&](int r, int c) {
            const bool dg = I0 + r == J0 + c;
            return (E)(weight(a[r][c], b[c][r], dg) - weight(b[c][r], a[r][c], dg));
        });
        if (I0 != J0)
            tio::store<E>(w, ldw, J0, I0, m, m, wv,
                          [&](int r, int c) { return (E)(weight(b[r][c], a[c][r], false) - weight(a[c][r], b[r][c], false)); });
        return;
    }
    // edges (I0 + r, J0 + c) into w; edges (I0 + c, J0 + r) into wt row J0 + r
    if (w) tio::store<E>(w, ldw, I0, J0, m, m, wv, [&](int r, int c) { return weight(a[r][c], b[c][r], I0 + r == J0 + c); });
    if (wt) tio::store<E>(wt, ldwt, J0, I0, m, m, wtv, [&](int r, int c) { return weight(a[c][r], b[r][c], I0 + c == J0 + r); });
    if (I0 == J0) return;
    // edges (J0 + r, I0 + c) into w; edges (J0 + c, I0 + r) into wt row I0 + r
    if (w) tio::store<E>(w, ldw, J0, I0, m, m, wv, [&](int r, int c) { return weight(b[r][c], a[c][r], false); });
    if (wt) tio::store<E>(wt, ldwt, I0, J0, m, m, wtv, [&](int r, int c) { return weight(b[c][r], a[r][c], false); });
}

// ------------------------------------------------------------------ sweeps
// NP widest-path problems from (to) one vertex s, side by side in one
// launch: problem q relaxes over the rows of A[q] and writes out[q].
template <typename E, int NP>
struct WidestArgs {
    sweep::Run<uint32_t, E, NP> run;
    int32_t m;
    int32_t s;   // source (target, with transposed weights)
    E *out[NP];  // m widths each, out[q][s] = 0
};

// x = MAX at s, 0 elsewhere; stamps 0; first frontier {s}; counters and
// barrier cleared.  A plain launch ahead of the sweeps, so that the sweeps
// need no barrier before their first step.
template <typename E, int NP>
__global__ __launch_bounds__(256) void k_widest_init(WidestArgs<E, NP> a) {
    const int32_t m = a.m;
    for (int q = 0; q < NP; ++q) {
        const sweep::Problem<uint32_t, E> &P = a.run.p[q];
        for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) {
            P.x[j] = j == a.s ? (uint32_t)max_value<E>() : 0u;
            P.stamp[j] = 0;
        }
        if (blockIdx.x == 0 && threadIdx.x < 4) P.count[threadIdx.x] = threadIdx.x == 0 ? 1 : 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) P.front[0][0] = a.s;
    }
    uint32_t *bar = reinterpret_cast<uint32_t *>(a.run.bar);
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < grid::BAR_WORDS; i += gridDim.x * 256) bar[i] = 0u;
}

// SIGNED: every problem's matrix holds signed weights S (int32); problem 0
// takes edge weights max(S, 0), problem 1 max(-S, 0) (|S| < 2^31).
template <typename E, int NP, bool SIGNED>
__global__ __launch_bounds__(256) void k_widest(WidestArgs<E, NP> a) {
    static_assert(!SIGNED || sizeof(E) == 4, "signed weights are int32");
    const int32_t m = a.m;
    const bool ok = sweep::run<uint32_t, E, NP>(
        a.run, m,
        [](int q, uint32_t xi, uint32_t e) {
            if constexpr (SIGNED) {
                const int32_t v = q ? -(int32_t)e : (int32_t)e;
                e = (uint32_t)max(v, 0);
            }
            return min(xi, e);
        },
        [](int32_t) { return true; });
    if (!ok) {
        if (threadIdx.x == 0) set_device_error(a.run.err, SCHULZE_EDEVICE);
        return;
    }
    for (int q = 0; q < NP; ++q)
        for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256)
            a.out[q][j] = j == a.s ? (E)0 : (E)a.run.p[q].x[j];
}

// ------------------------------------------------------------------ checks on the counts
// The same two widest-path problems straight from d: the weight
// w[i][j] = f(d[i][j], d[j][i]) is formed where it is used, so no weight
// matrix is written first.  A sweep whose frontiers (both directions
// together) hold at most m / CHECK_DENSE_RATIO vertices reads, for each
// frontier vertex v, row v of d as 16-byte vectors and column v one
// element per row: w[v][k] = f(d[v][k], d[k][v]) (source direction) and
// w[k][v] = f(d[k][v], d[v][k]) (target direction).  A sweep with larger
// frontiers relaxes every edge instead, in one pass over the 64 x 64 tile
// pairs (X, Y), (Y, X), X <= Y, of d, each read once: row x of a tile
// takes, over the tile's columns y,
//     source direction:  x0[x] <- max(x0[x], min(x0[y], w[y][x])),
//     target direction:  x1[x] <- max(x1[x], min(x1[y], w[x][y]))
// (relaxing rows outside the frontier changes nothing: every value is the
// width of some path).  A gathered column costs about a line per element,
// so the dense pass is the cheaper one beyond about m / 16 frontier rows.
constexpr int CHECK_DENSE_RATIO = 16;
constexpr int CHECK_ROW_LANES = 4;  // lanes per tile row (0.88 ms at m = 32768; eight: 0.96 ms)
constexpr int CHECK_RPT = CHECK_ROW_LANES * tio::T / 256;  // rows per thread: r + h * CHECK_ROW_STEP
constexpr int CHECK_ROW_STEP = tio::T / CHECK_RPT;

template <bool MARGIN>
__device__ __forceinline__ uint32_t edge_weight(int32_t a, int32_t b) {  // d[i][j] = a, d[j][i] = b
    return a > b ? (uint32_t)(MARGIN ? a - b : a) : 0u;
}

// Tile pair p (0 <= p < nb (nb + 1) / 2) as (X, Y), X <= Y, row by row:
// start(X) = X nb - X (X - 1) / 2 pairs come before row X.
__device__ inline void tile_pair(int64_t p, int32_t nb, int32_t &X, int32_t &Y) {
    auto start = [nb](int64_t r) { return r * nb - r * (r - 1) / 2; };
    const double b = (double)nb + 0.5;
    int32_t x = (int32_t)(b - sqrt(b * b - 2.0 * (double)p));
    x = x < 0 ? 0 : (x > nb - 1 ? nb - 1 : x);
    while (x > 0 && start(x) > p) --x;
    while (x + 1 < nb && start(x + 1) <= p) ++x;
    X = x;
    Y = x + (int32_t)(p - start(x));
}

// Append vertex j to a frontier list where `add` holds (all lanes of the
// wavefront take part).
__device__ inline void append(bool add, int32_t j, int32_t *cnt, int32_t *list) {
    const uint64_t bal = __ballot(add);
    if (!bal) return;
    const int lane = threadIdx.x & 63;
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(cnt, (int32_t)__popcll(bal));
    base = __shfl(base, 0);
    if (add) list[base + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = j;
}

// x[j] <- max(x[j], v); true if v raised it and j is not yet listed for
// sweep t + 1 (seen: a value x[j] held earlier in the sweep).
__device__ inline bool raise(uint32_t *x, int32_t *stamp, int32_t j, uint32_t v, uint32_t seen, int32_t t) {
    if (v <= seen || atomicMax(&x[j], v) >= v) return false;
    return atomicMax(&stamp[j], t + 1) < t + 1;
}

// Row r of a tile view (A[r][c] = d[x][y], B[c][r] = d[y][x], y the tile's
// column c): the lane's share of both directions' candidate values, with
// xc[q][c] = x_q[y] (0 past m).
template <typename E, bool MARGIN>
__device__ __forceinline__ void check_row(const E (*A)[tio::PITCH], const E (*B)[tio::PITCH],
                                          const uint32_t (*xc)[tio::T], int r, int g, uint32_t &v0, uint32_t &v1) {
    constexpr int V = 16 / (int)sizeof(E), KV = tio::T / (CHECK_ROW_LANES * V);
    for (int k = 0; k < KV; ++k)
        for (int u = 0; u < V; ++u) {
            const int c = k * CHECK_ROW_LANES * V + g * V + u;
            const int32_t a = (int32_t)A[r][c], b = (int32_t)B[c][r];
            v0 = max(v0, min(xc[0][c], edge_weight<MARGIN>(b, a)));
            v1 = max(v1, min(xc[1][c], edge_weight<MARGIN>(a, b)));
        }
}

// Both directions from (to) a.s over d (both problems' A = d), to the
// fixpoint, in one cooperative launch after k_widest_init.  VD: d is
// vector-aligned and m a multiple of the vector length.  Three workgroups
// per CU (registers capped accordingly; a few spill in the gather branch):
// 0.95 ms instead of 1.11 ms with two at m = 32768.
template <typename E, bool MARGIN, bool VD>
__global__ __launch_bounds__(256, 3) void k_check(WidestArgs<E, 2> a) {
    using sweep::CB;
    using sweep::CPL;
    __shared__ E ta[tio::T][tio::PITCH];      // ta[r][c] = d[X0 + r][Y0 + c]
    __shared__ E tb[tio::T][tio::PITCH];      // tb[r][c] = d[Y0 + r][X0 + c]
    __shared__ uint32_t xs[2][2][tio::T];     // xs[side][q][c] = x_q[(side ? Y0 : X0) + c], 0 past m
    __shared__ uint32_t part[4][CB];          // per-wavefront partial maxima of a column block
    const sweep::Run<uint32_t, E, 2> &R = a.run;
    const E *__restrict__ d = R.p[0].A;
    const int64_t ld = R.p[0].ld;
    const int32_t m = a.m, G = gridDim.x, g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *const x0 = R.p[0].x, *const x1 = R.p[1].x;
    int32_t *const st0 = R.p[0].stamp, *const st1 = R.p[1].stamp;
    // dense pass: tile pairs, CHECK_RPT rows per thread
    const int32_t nb = (m + tio::T - 1) / tio::T;
    const int64_t npairs = (int64_t)nb * (nb + 1) / 2;
    const int r = wave * (64 / CHECK_ROW_LANES) + lane / CHECK_ROW_LANES, gl = lane % CHECK_ROW_LANES;
    // gather: column blocks of both problems, a share of the frontier each
    const int32_t ncb = (m + CB - 1) / CB, nblk = 2 * ncb;
    const int32_t shares = G >= nblk ? G / nblk : 1;
    const bool gactive = g < nblk * shares;
    const int32_t blk = g % nblk, share = g / nblk, gq = blk / ncb, cb = blk % ncb;
    const int32_t blk0 = cb * CB, valid = m - blk0;
    for (int32_t t = 0;; ++t) {
        const int32_t n0 = __hip_atomic_load(R.p[0].count + t % 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t n1 = __hip_atomic_load(R.p[1].count + t % 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n0 == 0 && n1 == 0) break;
        if (t >= R.max_sweeps) {  // values only grow, so this cannot happen
            if (threadIdx.x == 0) set_device_error(R.err, SCHULZE_EDEVICE);
            return;
        }
        if (g == 0 && threadIdx.x == 0)
            for (int q = 0; q < 2; ++q) {
                // the list two sweeps ahead (read in the previous sweep, appended to in the next)
                R.p[q].count[(t + 2) % 3] = 0;
                if (R.p[q].count[t % 3]) ++R.p[q].count[3];
            }
        int32_t *const cn0 = R.p[0].count + (t + 1) % 3, *const cn1 = R.p[1].count + (t + 1) % 3;
        int32_t *const fn0 = R.p[0].front[(t + 1) & 1], *const fn1 = R.p[1].front[(t + 1) & 1];
        if ((int64_t)(n0 + n1) * CHECK_DENSE_RATIO > m) {
            // ---- dense pass over the tile pairs
            // A pair's two tiles and the 256 values of its rows and columns
            // (one per thread: side, direction, index) are loaded into
            // registers while the previous pair is worked on; the values may
            // be a pair old, which only delays a raise to the next sweep.
            tio::Regs<E> ga, gb;
            uint32_t xr = 0;
            const int xside = (threadIdx.x >> 7) & 1, xq = (threadIdx.x >> 6) & 1;
            auto fetch = [&](int32_t Xf, int32_t Yf) {
                tio::fetch<E, VD>(ga, d, ld, Xf * tio::T, Yf * tio::T, m, m);
                if (Xf != Yf) tio::fetch<E, VD>(gb, d, ld, Yf * tio::T, Xf * tio::T, m, m);
                const int32_t v = (xside ? Yf : Xf) * tio::T + lane;
                xr = v < m ? __hip_atomic_load((xq ? x1 : x0) + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
            };
            int64_t p = g;
            int32_t X = 0, Y = 0;
            if (p < npairs) {
                tile_pair(p, nb, X, Y);
                fetch(X, Y);
            }
            while (p < npairs) {
                const int32_t X0 = X * tio::T, Y0 = Y * tio::T;
                const bool diag = X == Y;
                __syncthreads();  // the previous pair's LDS reads are done
                tio::put<E>(ta, ga);
                if (!diag) tio::put<E>(tb, gb);
                xs[xside][xq][lane] = xr;
                const int64_t pn = p + G;
                int32_t Xn = 0, Yn = 0;
                if (pn < npairs) {  // in flight during the work below
                    tile_pair(pn, nb, Xn, Yn);
                    fetch(Xn, Yn);
                }
                __syncthreads();
                for (int side = 0; side < (diag ? 1 : 2); ++side) {
                    // side 0: rows of X over the columns of Y (X itself on the diagonal); side 1: rows of Y over X
                    const E(*A)[tio::PITCH] = side ? tb : ta;
                    const E(*B)[tio::PITCH] = diag ? ta : (side ? ta : tb);
                    const int cs = diag ? 0 : 1 - side;
                    const int32_t row0 = side ? Y0 : X0;
                    for (int h = 0; h < CHECK_RPT; ++h) {
                        const int rr = r + h * CHECK_ROW_STEP;
                        uint32_t v0 = 0, v1 = 0;
                        check_row<E, MARGIN>(A, B, xs[cs], rr, gl, v0, v1);
                        for (int off = 1; off < CHECK_ROW_LANES; off <<= 1) {
                            v0 = max(v0, (uint32_t)__shfl_xor((int)v0, off));
                            v1 = max(v1, (uint32_t)__shfl_xor((int)v1, off));
                        }
                        const int32_t row = row0 + rr;
                        const bool mine = gl == 0 && row < m;
                        const bool up0 = mine && raise(x0, st0, row, v0, xs[side][0][rr], t);
                        const bool up1 = mine && raise(x1, st1, row, v1, xs[side][1][rr], t);
                        append(up0, row, cn0, fn0);
                        append(up1, row, cn1, fn1);
                    }
                }
                p = pn;
                X = Xn;
                Y = Yn;
            }
        } else {
            // ---- gather: rows and columns of d for the frontier vertices
            const int32_t nf = gq ? n1 : n0;
            const int32_t *F = R.p[gq].front[t & 1];
            const uint32_t *xq = gq ? x1 : x0;
            uint32_t best[CPL] = {};
            if (gactive) {
                const bool full = VD && valid >= CB;
                for (int32_t qi = share * 4 + wave; qi < nf; qi += 4 * shares) {
                    const int32_t v = F[qi];
                    uint32_t row[CPL], col[CPL];
                    if (full)
                        sweep::load_row<E, true>(d + (int64_t)v * ld + blk0, valid, lane, row);
                    else
                        sweep::load_row<E, false>(d + (int64_t)v * ld + blk0, valid, lane, row);
                    for (int c = 0; c < CPL; ++c) {
                        const int32_t k = blk0 + sweep::lane_col<E>(lane, c);
                        col[c] = k < m ? (uint32_t)d[(int64_t)k * ld + v] : 0u;
                    }
                    const uint32_t xv = xq[v];
                    for (int c = 0; c < CPL; ++c) {
                        const uint32_t w = gq ? edge_weight<MARGIN>((int32_t)col[c], (int32_t)row[c])
                                              : edge_weight<MARGIN>((int32_t)row[c], (int32_t)col[c]);
                        best[c] = max(best[c], min(xv, w));
                    }
                }
                for (int c = 0; c < CPL; ++c) part[wave][sweep::lane_col<E>(lane, c)] = best[c];
            }
            __syncthreads();
            uint32_t *const xg = gq ? x1 : x0;
            int32_t *const sg = gq ? st1 : st0;
            for (int c = 0; c < CB / 256; ++c) {
                const int32_t jl = c * 256 + threadIdx.x, j = blk0 + jl;
                bool up = false;
                if (gactive && j < m) {
                    const uint32_t v = max(max(part[0][jl], part[1][jl]), max(part[2][jl], part[3][jl]));
                    up = raise(xg, sg, j, v, xg[j], t);
                }
                append(up, j, gq ? cn1 : cn0, gq ? fn1 : fn0);
            }
        }
        if (!grid::grid_sync(R.bar, R.spin_limit)) {
            if (threadIdx.x == 0) set_device_error(R.err, SCHULZE_EDEVICE);
            return;
        }
    }
    for (int q = 0; q < 2; ++q)
        for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256)
            a.out[q][j] = j == a.s ? (E)0 : (E)R.p[q].x[j];
}

// ------------------------------------------------------------------ verdict
// out[0] = 1 if c is a winner; out[1] = number of candidates beating c;
// out[2] = a beater (highest score, or widest margin p(x,c) - p(c,x) when
// no scores are given; ties -> lowest id) or -1; out[3] = number of x != c
// tied with c (p(c,x) = p(x,c)).  tied[] (optional) lists them.
constexpr int TALLY_THREADS = 1024;
template <typename E>
__global__ __launch_bounds__(TALLY_THREADS) void k_verdict(const E *__restrict__ from, const E *__restrict__ to,
                                                             int32_t m, int32_t c, const float *__restrict__ score,
                                                             int32_t *out, int32_t *tied) {
    // one workgroup; counts and the tied list per wavefront (ballots), the
    // best beater as a wavefront maximum, then one LDS atomic each
    __shared__ int32_t nbeat, ntie;
    __shared__ unsigned long long best;
    if (threadIdx.x == 0) {
        nbeat = 0;
        ntie = 0;
        best = 0ull;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    unsigned long long mine = 0ull;
    int32_t beats = 0;
    // uniform trip count (the ballots below see every lane); four
    // candidates per thread loaded together
    for (int32_t x0 = 0; x0 < m; x0 += 4 * TALLY_THREADS) {
        E fv[4], tv[4];
        for (int u = 0; u < 4; ++u) {
            const int32_t x = x0 + u * TALLY_THREADS + (int32_t)threadIdx.x;
            const int32_t xc = x < m ? x : 0;
            fv[u] = from[xc];
            tv[u] = to[xc];
        }
        for (int u = 0; u < 4; ++u) {
            const int32_t x = x0 + u * TALLY_THREADS + (int32_t)threadIdx.x;
            const bool in = x < m && x != c;
            const E f = fv[u], t = tv[u];
            const bool beat = in && t > f, tie = in && t == f;
            if (beat) {
                ++beats;
                // key: larger is better; ids ascending on ties
                uint32_t hi;
                if (score) {
                    const uint32_t bits = __float_as_uint(score[x]);
                    hi = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);  // order-preserving
                } else {
                    hi = (uint32_t)(t - f);
                }
                const unsigned long long key = ((unsigned long long)hi << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)x);
                mine = key > mine ? key : mine;
            }
            const uint64_t bal = __ballot(tie);
            if (bal) {
                int32_t base = 0;
                if (lane == 0) base = atomicAdd(&ntie, (int32_t)__popcll(bal));
                base = __shfl(base, 0);
                if (tie && tied) tied[base + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = x;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off);
        mine = o > mine ? o : mine;
        beats += __shfl_xor(beats, off);
    }
    if (lane == 0) {
        atomicMax(&best, mine);
        atomicAdd(&nbeat, beats);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = nbeat == 0 ? 1 : 0;
        out[1] = nbeat;
        out[2] = nbeat ? (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull)) : -1;
        out[3] = ntie;
    }
}

// Scratch of one launch of np widest-path problems: per problem values,
// stamps, two frontier lists and counters; then the barrier.
size_t widest_scratch_bytes(int32_t m, int np) {
    const size_t v = round_up(sizeof(uint32_t) * (size_t)m, 256);
    return (size_t)np * (4 * v + 256) + round_up(grid::BAR_BYTES, 256);
}

// Widest paths from src over the rows of A[q] (q < NP) into out[q], with
// the sweep state in `base` (widest_scratch_bytes(m, NP) bytes of device
// memory, all of it set by the init launch before it is read).  `timed`
// brackets both launches with the context's timing events.  SIGNED: A[q]
// hold signed weights (see k_widest).
template <typename E, int NP, bool SIGNED = false>
int widest_in(schulze_ctx *ctx, hipStream_t s, const E *const (&A)[NP], const int64_t (&ld)[NP], int32_t m,
              int32_t src, E *const (&out)[NP], char *base, bool timed) {
    const size_t v = round_up(sizeof(uint32_t) * (size_t)m, 256);
    WidestArgs<E, NP> a;
    for (int q = 0; q < NP; ++q) {
        char *p = base + (size_t)q * (4 * v + 256);
        sweep::Problem<uint32_t, E> &P = a.run.p[q];
        P.A = A[q];
        P.ld = ld[q];
        P.vec = sweep::vec_ok<E>(A[q], ld[q]) ? 1 : 0;
        P.x = reinterpret_cast<uint32_t *>(p);
        P.stamp = reinterpret_cast<int32_t *>(p + v);
        P.front[0] = reinterpret_cast<int32_t *>(p + 2 * v);
        P.front[1] = reinterpret_cast<int32_t *>(p + 3 * v);
        P.count = reinterpret_cast<int32_t *>(p + 4 * v);
        a.out[q] = out[q];
    }
    a.run.max_sweeps = ctx->sweep_max_sweeps > 0 ? ctx->sweep_max_sweeps : m + 1;
    a.run.bar = reinterpret_cast<GridBar *>(base + (size_t)NP * (4 * v + 256));
    a.run.err = ctx->err;
    a.run.spin_limit = ctx->sweep_spin_limit > 0 ? ctx->sweep_spin_limit : SWEEP_SPIN_LIMIT;
    a.m = m;
    a.s = src;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_widest<E, NP, SIGNED>, 256, 0) != hipSuccess ||
        per_cu < 1)
        return SCHULZE_EDEVICE;
    const int64_t G = sweep::grid_size(m, NP, (int64_t)ctx->num_cus * std::min(per_cu, 2));
    int tok = -1;
    if (timed) timing_begin(ctx, K_WIDEST, s, &tok);
    k_widest_init<E, NP><<<dim3((unsigned)std::min<int64_t>(ceil_div(m, 256), 1024)), dim3(256), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    void *args[] = {&a};
    if (e == hipSuccess)
        e = hipLaunchCooperativeKernel((const void *)k_widest<E, NP, SIGNED>, dim3((unsigned)G), dim3(256), args, 0,
                                       s);
    if (timed) timing_end(ctx, tok, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SCHULZE_EDEVICE;
    }
    return SCHULZE_OK;
}

template <typename E>
int widest(schulze_ctx *ctx, hipStream_t s, const E *w, int64_t ldw, int32_t m, int32_t src, E *out) {
    int rc = ws_reserve(ctx, WS_VERIFY, widest_scratch_bytes(m, 1));
    if (rc != SCHULZE_OK) return rc;
    const E *const A[1] = {w};
    const int64_t ld[1] = {ldw};
    E *const o[1] = {out};
    return widest_in<E, 1>(ctx, s, A, ld, m, src, o, static_cast<char *>(ctx->ws[WS_VERIFY]), true);
}

// Both widest-path directions (one launch) and the verdict, with the sweep
// state in base (nullptr: the context's workspace).  SIGNED: w = wt = the
// signed weights.
template <typename E, bool SIGNED = false>
int verify_all(schulze_ctx *ctx, hipStream_t s, const E *w, int64_t ldw, const E *wt, int64_t ldwt, int32_t m,
               int32_t cand, const float *score, E *p_from, E *p_to, int32_t *verdict, int32_t *tied, char *base) {
    int rc;
    const E *const A[2] = {w, wt};
    const int64_t ld[2] = {ldw, ldwt};
    E *const out[2] = {p_from, p_to};
    if (base) {
        if ((rc = widest_in<E, 2, SIGNED>(ctx, s, A, ld, m, cand, out, base, false)) != SCHULZE_OK) return rc;
        k_verdict<E><<<dim3(1), dim3(TALLY_THREADS), 0, s>>>(p_from, p_to, m, cand, score, verdict, tied);
        return launch_status();
    }
    if ((rc = ws_reserve(ctx, WS_VERIFY, widest_scratch_bytes(m, 2))) != SCHULZE_OK) return rc;
    if ((rc = widest_in<E, 2, SIGNED>(ctx, s, A, ld, m, cand, out, static_cast<char *>(ctx->ws[WS_VERIFY]),
                                      true)) != SCHULZE_OK)
        return rc;
    SCHULZE_LAUNCH(ctx, K_VERDICT, s,
                   k_verdict<E><<<dim3(1), dim3(TALLY_THREADS), 0, s>>>(p_from, p_to, m, cand, score, verdict, tied));
    return SCHULZE_OK;
}

// The exact check of cand from d (k_check) and its verdict.
template <typename E, bool MARGIN, bool VD>
int check_counts_as(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int32_t cand,
                    const float *score, E *p_from, E *p_to, int32_t *verdict, int32_t *tied) {
    int rc = ws_reserve(ctx, WS_VERIFY, widest_scratch_bytes(m, 2));
    if (rc != SCHULZE_OK) return rc;
    char *base = static_cast<char *>(ctx->ws[WS_VERIFY]);
    const size_t v = round_up(sizeof(uint32_t) * (size_t)m, 256);
    WidestArgs<E, 2> a;
    for (int q = 0; q < 2; ++q) {
        char *p = base + (size_t)q * (4 * v + 256);
        sweep::Problem<uint32_t, E> &P = a.run.p[q];
        P.A = d;
        P.ld = ldd;
        P.vec = VD ? 1 : 0;
        P.x = reinterpret_cast<uint32_t *>(p);
        P.stamp = reinterpret_cast<int32_t *>(p + v);
        P.front[0] = reinterpret_cast<int32_t *>(p + 2 * v);
        P.front[1] = reinterpret_cast<int32_t *>(p + 3 * v);
        P.count = reinterpret_cast<int32_t *>(p + 4 * v);
    }
    a.out[0] = p_from;
    a.out[1] = p_to;
    a.run.max_sweeps = ctx->sweep_max_sweeps > 0 ? ctx->sweep_max_sweeps : m + 1;
    a.run.bar = reinterpret_cast<GridBar *>(base + 2 * (4 * v + 256));
    a.run.err = ctx->err;
    a.run.spin_limit = ctx->sweep_spin_limit > 0 ? ctx->sweep_spin_limit : SWEEP_SPIN_LIMIT;
    a.m = m;
    a.s = cand;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_check<E, MARGIN, VD>, 256, 0) != hipSuccess ||
        per_cu < 1)
        return SCHULZE_EDEVICE;
    // enough workgroups for the tile pairs of the dense pass and for every
    // column block of both gather problems (cap >= 128 >= 2 ceil(m / 1024))
    const int64_t nb = ceil_div(m, 64);
    const int64_t want = std::max<int64_t>(sweep::grid_size(m, 2, INT64_MAX), nb * (nb + 1) / 2);
    const int64_t G = std::min<int64_t>((int64_t)ctx->num_cus * std::min(per_cu, 3), want);
    int tok = -1;
    timing_begin(ctx, K_WIDEST, s, &tok);
    k_widest_init<E, 2><<<dim3((unsigned)std::min<int64_t>(ceil_div(m, 256), 1024)), dim3(256), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    void *args[] = {&a};
    if (e == hipSuccess)
        e = hipLaunchCooperativeKernel((const void *)k_check<E, MARGIN, VD>, dim3((unsigned)G), dim3(256), args, 0,
                                       s);
    timing_end(ctx, tok, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SCHULZE_EDEVICE;
    }
    SCHULZE_LAUNCH(ctx, K_VERDICT, s,
                   k_verdict<E><<<dim3(1), dim3(TALLY_THREADS), 0, s>>>(p_from, p_to, m, cand, score, verdict, tied));
    return SCHULZE_OK;
}

template <typename E>
int check_counts(schulze_ctx *ctx, hipStream_t s, const E *d, int64_t ldd, int32_t m, int mode, int32_t cand,
                 const float *score, E *p_from, E *p_to, int32_t *verdict, int32_t *tied) {
    constexpr int V = 16 / (int)sizeof(E);
    const bool vd = tio::vec_ok<E>(d, ldd) && m % V == 0;
    if (mode == SCHULZE_MARGIN)
        return vd ? check_counts_as<E, true, true>(ctx, s, d, ldd, m, cand, score, p_from, p_to, verdict, tied)
                  : check_counts_as<E, true, false>(ctx, s, d, ldd, m, cand, score, p_from, p_to, verdict, tied);
    return vd ? check_counts_as<E, false, true>(ctx, s, d, ldd, m, cand, score, p_from, p_to, verdict, tied)
              : check_counts_as<E, false, false>(ctx, s, d, ldd, m, cand, score, p_from, p_to, verdict, tied);
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
    if (widest_scratch_bytes(m, 2) > VERIFY_SCRATCH_BYTES) return SCHULZE_EUNSUPPORTED;
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

extern "C" int schulze_verify_counts(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                                     int dtype, int mode, int32_t cand, const float *score, void *p_from,
                                     void *p_to, int32_t *verdict, int32_t *tied) {
    int rc = check_square(ctx, d, ldd, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (!p_from || !p_to || !verdict || cand < 0 || cand >= m) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SCHULZE_U16) {
        using E = uint16_t;
        return check_counts<E>(ctx, s, static_cast<const E *>(d), ldd, m, mode, cand, score, static_cast<E *>(p_from),
                               static_cast<E *>(p_to), verdict, tied);
    }
    using E = int32_t;
    return check_counts<E>(ctx, s, static_cast<const E *>(d), ldd, m, mode, cand, score, static_cast<E *>(p_from),
                           static_cast<E *>(p_to), verdict, tied);
}

int signed_weights(schulze_ctx *ctx, hipStream_t s, const int32_t *d, int64_t ldd, int32_t m, int mode, int32_t *S,
                   int64_t lds) {
    const int vec = (tio::vec_ok<int32_t>(d, ldd) ? 1 : 0) | (tio::vec_ok<int32_t>(S, lds) ? 2 : 0);
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(m, 64));
    SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                   k_weights_pair<int32_t, true><<<grid, dim3(256), 0, s>>>(d, ldd, m, mode, S, lds, nullptr, 0, vec));
    return SCHULZE_OK;
}

// Internal: schulze_verify over signed weights sw = w - w^T (int32, pitch
// ld; device pointers, m <= 65535, cand < m, checked by the caller).
int verify_signed(schulze_ctx *ctx, hipStream_t s, const int32_t *sw, int64_t ld, int32_t m, int32_t cand,
                  const float *score, int32_t *p_from, int32_t *p_to, int32_t *verdict, int32_t *tied) {
    return verify_all<int32_t, true>(ctx, s, sw, ld, sw, ld, m, cand, score, p_from, p_to, verdict, tied, nullptr);
}
