// Pairwise preference counts d[x][y] (Section 2.1: profile of weak orders).
//
// d[x][y] is the total weight of voters who list x and list y later or not
// at all.  Ballots are split by a scan into full rankings (at least m-1
// listed candidates) and truncated ballots, which take different routes:
//
//  * Position counting.  The rank of every candidate is scattered into a
//    position array, two voters per 32-bit word (low half: one voter, high
//    half: the next).  For one (x, y) pair and one voter, the 16-bit
//    difference t = (pos(x) - pos(y)) mod 2^16 equals
//    pos(x) - pos(y) + 2^16 [pos(x) < pos(y)], so summed over voters
//        sum t = Sx - Sy + 2^16 * #(x before y),
//    where Sx is the sum of x's positions.  One v_pk_sub_u16 yields t for two
//    voters and one v_dot2_u32_u16 adds both halves into a 32-bit
//    accumulator: one VALU lane-op per comparison.  The count is
//    (acc - Sx + Sy) >> 16, exact while fewer than 2^16 voters are summed.
//    - Full rankings have no ties, so only tiles with x-block <= y-block are
//      counted and d[y][x] = voters - d[x][y].
//    - Truncated ballots are counted the same way over the candidates U that
//      any truncated ballot lists (unlisted candidates share one sentinel
//      position, so ties count for neither side), over all ordered tiles.
//      One extra always-sentinel column gives R[x], the number of truncated
//      ballots listing x, and d[x][y] = R[x] for x in U, y outside U.
//  * Pair scattering, for truncated ballots when U is large: d[x][y] =
//    R[x] - C[y][x], where C[y][x] is the weight of ballots listing y before
//    x; the listed pairs are scattered with atomics.
// A small decision kernel picks the cheaper truncated route on the device.
// Everything accumulates into one m x m uint32 matrix that a final pass
// completes and converts to the output dtype.
#include "internal.h"

namespace {

constexpr int CT = 128;           // count tile (candidates per side)
constexpr int VC = 32;            // voter pairs per staged chunk
constexpr int CNT_THREADS = 256;
constexpr int SEG_PAIRS = 32767;  // at most 65534 voters per exact segment
constexpr int SEGC = SEG_PAIRS / VC;
constexpr int SCATTER_CH = 8192;  // columns per LDS chunk of the scatters
constexpr int LONG_CHUNK = 32;    // ballots per workgroup of the long-row scan
constexpr int SHORT_PER_WAVE = 8; // steps (groups of ballots) per wavefront of the short-row scan
constexpr int NPART = 64;         // partial sums of the pair-scattering cost
constexpr uint16_t UNSET = 0xFFFF;

enum { MODE_SPARSE = 0, MODE_DENSE_U = 1 };

typedef __attribute__((ext_vector_type(2))) unsigned short us2;

// Workspace views (WS_BALLOT_META).
struct Meta {
    int32_t *ctr;            // [0] full rankings [1] truncated ballots [2] route
                             // [3] |U| [4] U-space pitch [32..33] total voter
                             // weight (64 bits) [34] its workgroups done
    unsigned long long *k2;  // NPART partial sums of k(k-1)/2 over truncated ballots
    int32_t *len;            // listed length per ballot
    int32_t *full_src;       // slot -> ballot of a full ranking
    int32_t *trunc_src;      // slot -> ballot of a truncated ballot
    uint8_t *in_u;           // candidate listed by some truncated ballot
    int32_t *ulist;          // U-space index -> candidate
    int32_t *umap;           // candidate -> U-space index or -1
};

// Ballot entry idx, -1 for padding.  The id type is a template parameter:
// a branch on it at every load made each load wait for the one before.
template <bool I32>
__device__ inline uint32_t load_raw(const void *ballots, int64_t idx) {
    if constexpr (I32)
        return static_cast<const uint32_t *>(ballots)[idx];
    else
        return static_cast<const uint16_t *>(ballots)[idx];
}
template <bool I32>
__device__ inline int32_t raw_id(uint32_t raw) {
    if constexpr (I32)
        return (int32_t)raw < 0 ? -1 : (int32_t)raw;
    else
        return raw == 0xFFFFu ? -1 : (int32_t)raw;
}
template <bool I32>
__device__ inline int32_t read_id(const void *ballots, int64_t idx) {
    return raw_id<I32>(load_raw<I32>(ballots, idx));
}

// ------------------------------------------------------------------ scan
// Listed length, id range check, full/truncated split (slots reserved once
// per workgroup), candidates listed by truncated ballots, and the pair count
// of the truncated ballots.
__device__ inline void record_ballots(Meta meta, int nf, const int32_t *lf, int nt, const int32_t *lt) {
    __shared__ int32_t base_f, base_t;
    if (threadIdx.x == 0) {
        base_f = nf ? atomicAdd(&meta.ctr[0], nf) : 0;
        base_t = nt ? atomicAdd(&meta.ctr[1], nt) : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nf; i += blockDim.x) meta.full_src[base_f + i] = lf[i];
    for (int i = threadIdx.x; i < nt; i += blockDim.x) meta.trunc_src[base_t + i] = lt[i];
}

// Long rows: one workgroup walks LONG_CHUNK ballots.
template <bool I32>
__global__ __launch_bounds__(256) void k_scan_long(const void *__restrict__ ballots, int64_t n, int32_t L,
                                                   int32_t m, Meta meta, int32_t *err) {
    __shared__ int32_t first_pad;
    __shared__ int32_t lf[LONG_CHUNK], lt[LONG_CHUNK];
    __shared__ int32_t nf, nt;
    const int64_t v0 = (int64_t)blockIdx.x * LONG_CHUNK;
    if (threadIdx.x == 0) nf = nt = 0;
    bool bad = false;
    unsigned long long k2 = 0;
    for (int q = 0; q < LONG_CHUNK; ++q) {
        const int64_t v = v0 + q;
        if (v >= n) break;
        __syncthreads();
        if (threadIdx.x == 0) first_pad = L;
        __syncthreads();
        const int64_t base = v * (int64_t)L;
        for (int t = threadIdx.x; t < L; t += 256)
            if (read_id<I32>(ballots, base + t) < 0) {
                atomicMin(&first_pad, t);
                break;
            }
        __syncthreads();
        const int k = first_pad;
        const bool trunc = k < m - 1;
        for (int t = threadIdx.x; t < k; t += 256) {
            const int32_t c = read_id<I32>(ballots, base + t);
            if (c >= m)
                bad = true;
            else if (trunc)
                meta.in_u[c] = 1;
        }
        if (threadIdx.x == 0) {
            meta.len[v] = k;
            if (trunc) {
                lt[nt++] = (int32_t)v;
                k2 += (unsigned long long)k * (k - 1) / 2;
            } else {
                lf[nf++] = (int32_t)v;
            }
        }
    }
    if (bad) set_device_error(err, SCHULZE_EBALLOT);
    if (threadIdx.x == 0 && k2) atomicAdd(&meta.k2[blockIdx.x % NPART], k2);
    __syncthreads();
    record_ballots(meta, nf, lf, nt, lt);
}

// Long rows of uint16 ids (L a multiple of 8, 16-byte aligned rows): one
// wavefront per ballot, eight ids per 16-byte load; the first padding entry
// is a wavefront minimum, so no workgroup barrier is needed per ballot.  The
// full and truncated lists keep ballot order, as in k_scan_long.
__global__ __launch_bounds__(256) void k_scan_long_vec(const uint16_t *__restrict__ ballots, int64_t n, int32_t L,
                                                       int32_t m, Meta meta, int32_t *err) {
    __shared__ int32_t lf[LONG_CHUNK], lt[LONG_CHUNK];
    __shared__ uint8_t kind[LONG_CHUNK];  // 0 none, 1 full, 2 truncated
    __shared__ int32_t nf, nt;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t v0 = (int64_t)blockIdx.x * LONG_CHUNK;
    const int32_t L8 = L / 8;
    bool bad = false;
    unsigned long long k2 = 0;
    for (int q = wave; q < LONG_CHUNK; q += 4) {
        const int64_t v = v0 + q;
        if (v >= n) {
            if (lane == 0) kind[q] = 0;
            continue;
        }
        const uint4 *row = reinterpret_cast<const uint4 *>(ballots + v * (int64_t)L);
        int32_t first = L;
        for (int32_t j = lane; j < L8; j += 64) {
            const uint4 x = row[j];
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
            for (int e = 7; e >= 0; --e) {  // the lowest padding index of the eight wins
                const uint32_t raw = (e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xFFFFu);
                if (raw == 0xFFFFu) first = min(first, 8 * j + e);
            }
        }
        for (int off = 32; off >= 1; off >>= 1) first = min(first, __shfl_xor(first, off));
        const int32_t k = first;
        const bool trunc = k < m - 1;
        for (int32_t j = lane; 8 * j < k; j += 64) {
            const uint4 x = row[j];
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
            for (int e = 0; e < 8; ++e) {
                if (8 * j + e >= k) break;
                const int32_t c = (int32_t)((e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xFFFFu));
                if (c >= m)
                    bad = true;
                else if (trunc)
                    meta.in_u[c] = 1;
            }
        }
        if (lane == 0) {
            meta.len[v] = k;
            kind[q] = trunc ? 2 : 1;
            if (trunc) k2 += (unsigned long long)k * (k - 1) / 2;
        }
    }
    if (bad) set_device_error(err, SCHULZE_EBALLOT);
    if (lane == 0 && k2) atomicAdd(&meta.k2[blockIdx.x % NPART], k2);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t a = 0, b = 0;
        for (int q = 0; q < LONG_CHUNK; ++q) {
            if (kind[q] == 1) lf[a++] = (int32_t)(v0 + q);
            if (kind[q] == 2) lt[b++] = (int32_t)(v0 + q);
        }
        nf = a;
        nt = b;
    }
    __syncthreads();
    record_ballots(meta, nf, lf, nt, lt);
}

// Short rows (L <= 64): a wavefront takes 64 / L ballots at once (at most
// SHORT_BPW), one lane per entry, SHORT_PER_WAVE such steps with all their
// loads issued first, SHORT_ROUNDS times; a ballot's listed length is the
// first padding lane of its group (a wavefront ballot).  (More ballots per
// workgroup mean fewer list reservations on the two shared counters.)
constexpr int SHORT_BPW = 4;
constexpr int SHORT_ROUNDS = 4;
constexpr int32_t SEEN_BITS = 65536;
template <bool I32>
__global__ __launch_bounds__(256) void k_scan_short(const void *__restrict__ ballots, int64_t n, int32_t L,
                                                    int32_t m, Meta meta, int32_t *err) {
    constexpr int PER_WG = 4 * SHORT_PER_WAVE * SHORT_BPW * SHORT_ROUNDS;
    __shared__ int32_t lf[PER_WG], lt[PER_WG];
    __shared__ int32_t nf, nt;
    // candidates listed by this workgroup's truncated ballots, as bits (for
    // m <= SEEN_BITS; else marked in meta.in_u at once): one store per
    // candidate and workgroup at the end instead of a read of in_u at every
    // entry, which made each step wait for memory
    __shared__ uint32_t seen[SEEN_BITS / 32];
    const bool use_seen = m <= SEEN_BITS;
    if (threadIdx.x == 0) nf = nt = 0;
    if (use_seen)
        for (int32_t w = threadIdx.x; w < (m + 31) / 32; w += 256) seen[w] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t bpw = min(SHORT_BPW, 64 / L);
    const int32_t sub = lane / L, t = lane - sub * L;
    const bool lane_ok = sub < bpw;
    const uint64_t group_bits = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
    bool bad = false;
    unsigned long long k2 = 0;
    for (int round = 0; round < SHORT_ROUNDS; ++round) {
        const int64_t v0 = (((int64_t)blockIdx.x * SHORT_ROUNDS + round) * 4 + wave) * SHORT_PER_WAVE * bpw;
        int32_t c[SHORT_PER_WAVE];
        for (int q = 0; q < SHORT_PER_WAVE; ++q) {  // every load first
            const int64_t v = v0 + (int64_t)q * bpw + sub;
            // (every lane loads: a load under a condition is waited for inside it)
            c[q] = (int32_t)load_raw<I32>(ballots, lane_ok && v < n ? v * L + t : 0);
        }
        for (int q = 0; q < SHORT_PER_WAVE; ++q) {
            const int64_t v = v0 + (int64_t)q * bpw + sub;
            c[q] = lane_ok && v < n ? raw_id<I32>((uint32_t)c[q]) : -2;
        }
        for (int q = 0; q < SHORT_PER_WAVE; ++q) {
            const int64_t v = v0 + (int64_t)q * bpw + sub;
            const uint64_t pad = __ballot(c[q] < 0);  // -1 padding, -2 no ballot
            const uint64_t mine = lane_ok ? (pad >> (sub * L)) & group_bits : group_bits;
            const int k = mine ? (int)__builtin_ctzll(mine) : L;
            const bool live = lane_ok && v < n;
            const bool trunc = k < m - 1;
            if (live && t < k) {
                if (c[q] >= m) {
                    bad = true;
                } else if (trunc) {
                    if (use_seen) {
                        const uint32_t bit = 1u << (c[q] & 31);
                        if (!(seen[c[q] >> 5] & bit)) atomicOr(&seen[c[q] >> 5], bit);
                    } else if (!meta.in_u[c[q]]) {  // a read first: frequent candidates are set once per cache
                        meta.in_u[c[q]] = 1;
                    }
                }
            }
            if (live && t == 0) {
                meta.len[v] = k;
                if (trunc) {
                    lt[atomicAdd(&nt, 1)] = (int32_t)v;
                    k2 += (unsigned long long)k * (k - 1) / 2;
                } else {
                    lf[atomicAdd(&nf, 1)] = (int32_t)v;
                }
            }
        }
    }
    if (__ballot(bad) && lane == 0) set_device_error(err, SCHULZE_EBALLOT);
    for (int off = 32; off >= 1; off >>= 1) k2 += __shfl_xor(k2, off);
    if (lane == 0 && k2) atomicAdd(&meta.k2[(blockIdx.x * 4 + wave) % NPART], k2);
    __syncthreads();
    if (use_seen)
        for (int32_t c = threadIdx.x; c < m; c += 256)
            if ((seen[c >> 5] >> (c & 31)) & 1u) meta.in_u[c] = 1;
    record_ballots(meta, nf, lf, nt, lt);
}

// ------------------------------------------------------------------ route decision
// One workgroup: U-space compaction (prefix sum over candidates) and the
// choice between the dense route over U and pair scattering for truncated
// ballots.  Costs: dense ~ (n_T / 2) * pitch^2 lane-ops, pair counting
// ~ sum k(k-1)/2 pairs, a pair charged as pair_cost lane-ops (about the
// measured ratio of the two rates on MI355X: 1024 for device-wide atomics,
// 512 for the bucketed count).
constexpr double ATOMIC_PAIR_COST = 1024.0;
constexpr double BUCKETED_PAIR_COST = 512.0;

constexpr int ROUTE_THREADS = 1024;
constexpr int ROUTE_VEC = 4;  // 16-byte groups of flags per thread (m <= 65536)
__global__ __launch_bounds__(ROUTE_THREADS) void k_route(int32_t m, Meta meta, int weighted, int64_t cap_words,
                                                         double pair_cost) {
    __shared__ int32_t part[ROUTE_THREADS];
    // A thread takes consecutive flags (0 or 1 bytes; zero past m up to the
    // next 16 bytes), as ROUTE_VEC 16-byte loads issued together (a byte at
    // a time waited for memory at every flag), else one byte at a time.
    const bool vec = m <= ROUTE_THREADS * 16 * ROUTE_VEC;
    const int32_t groups = (m + 15) / 16;
    const int32_t gper = (groups + ROUTE_THREADS - 1) / ROUTE_THREADS;
    const int32_t g0 = (int32_t)threadIdx.x * gper;
    const int32_t per = vec ? 16 * gper : (m + ROUTE_THREADS - 1) / ROUTE_THREADS;
    const int32_t c0 = min(m, (int32_t)threadIdx.x * per), c1 = min(m, c0 + per);
    uint4 f[ROUTE_VEC];
    int32_t cnt = 0;
    if (vec) {
        const uint4 *in4 = reinterpret_cast<const uint4 *>(meta.in_u);
        for (int k = 0; k < ROUTE_VEC; ++k) f[k] = in4[k < gper && g0 + k < groups ? g0 + k : 0];
        for (int k = 0; k < ROUTE_VEC; ++k) {
            if (!(k < gper && g0 + k < groups)) f[k] = make_uint4(0u, 0u, 0u, 0u);
            cnt += __popc(f[k].x) + __popc(f[k].y) + __popc(f[k].z) + __popc(f[k].w);
        }
    } else {
        for (int32_t c = c0; c < c1; ++c) cnt += meta.in_u[c] ? 1 : 0;
    }
    part[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < ROUTE_THREADS; off <<= 1) {  // inclusive scan
        const int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t idx = part[threadIdx.x] - cnt;
    auto place = [&](int32_t c, bool in) {
        if (in) {
            meta.ulist[idx] = c;
            meta.umap[c] = idx++;
        } else {
            meta.umap[c] = -1;
        }
    };
    if (vec) {
        for (int k = 0; k < ROUTE_VEC; ++k) {
            const uint32_t w[4] = {f[k].x, f[k].y, f[k].z, f[k].w};
            for (int e = 0; e < 16; ++e) {
                const int32_t c = 16 * (g0 + k) + e;
                if (k < gper && c < m) place(c, (w[e >> 2] >> (8 * (e & 3))) & 1u);
            }
        }
    } else {
        for (int32_t c = c0; c < c1; ++c) place(c, meta.in_u[c] != 0);
    }
    if (threadIdx.x == 0) {
        const int32_t nu = part[ROUTE_THREADS - 1];
        const int32_t pitch = (nu + 1 + CT - 1) / CT * CT;  // room for one sentinel column
        const int64_t n_t = meta.ctr[1];
        unsigned long long k2 = 0;
        for (int i = 0; i < NPART; ++i) k2 += meta.k2[i];
        const int64_t pairs = (n_t + 1) / 2;
        const double dense = (double)pairs * (double)pitch * (double)pitch;
        const bool fits = pairs * (int64_t)pitch <= cap_words;
        const bool use_dense = !weighted && fits && n_t > 0 && dense <= pair_cost * (double)k2;
        meta.ctr[2] = use_dense ? MODE_DENSE_U : MODE_SPARSE;
        meta.ctr[3] = nu;
        meta.ctr[4] = pitch;
    }
}

// ------------------------------------------------------------------ scatters
// A workgroup per voter pair q (grid-stride over the pairs): positions of slots 2q (low half) and
// 2q+1 (high half; 0 for the missing partner of an odd count), staged in
// LDS in chunks of SCATTER_CH columns and written as rows of `pitch` words.
// A ballot lists distinct candidates iff its entries leave exactly
// (columns - listed) positions unset; anything else is a repeated id.
template <bool FULL, bool I32>
__global__ __launch_bounds__(256) void k_scatter(const void *__restrict__ ballots, int32_t L, int32_t m,
                                                 int32_t full_pitch, Meta meta, uint32_t *__restrict__ pos,
                                                 int32_t *err) {
    __shared__ uint16_t buf[2 * SCATTER_CH];
    __shared__ int32_t unset_cnt[2];
    const int32_t count = FULL ? meta.ctr[0] : meta.ctr[1];
    if (!FULL && meta.ctr[2] != MODE_DENSE_U) return;
    for (int64_t q = blockIdx.x; 2 * q < count; q += gridDim.x) {
    const int32_t pitch = FULL ? full_pitch : meta.ctr[4];
    const int32_t ncols = FULL ? m : meta.ctr[3];  // real columns: candidates or U
    const int32_t *srcs = FULL ? meta.full_src : meta.trunc_src;
    const bool has_hi = 2 * q + 1 < count;
    const int32_t src[2] = {srcs[2 * q], has_hi ? srcs[2 * q + 1] : -1};
    // 16-byte ballot reads (uint16 ids, rows 16-byte aligned) and position
    // stores (rows and chunks in multiples of four words)
    const bool vec16 = !I32 && (L % 8) == 0 && (reinterpret_cast<uintptr_t>(ballots) % 16) == 0;
    const bool vec_out = (pitch % 4) == 0 && (reinterpret_cast<uintptr_t>(pos) % 16) == 0;
    __syncthreads();  // the previous pair's counts have been read
    if (threadIdx.x < 2) unset_cnt[threadIdx.x] = 0;
    for (int32_t c0 = 0; c0 < pitch; c0 += SCATTER_CH) {
        const int32_t cn = min(SCATTER_CH, pitch - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < 2 * cn; i += 256) buf[i] = UNSET;
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            if (src[h] < 0) continue;
            const int32_t k = meta.len[src[h]];
            const int64_t base = (int64_t)src[h] * L;
            auto place = [&](int32_t t, int32_t id) {
                if (id < 0 || id >= m) return;  // reported by the scan
                const int32_t col = FULL ? id : meta.umap[id];
                if (col >= c0 && col < c0 + cn) buf[2 * (col - c0) + h] = (uint16_t)t;
            };
            if (vec16) {
                // eight uint16 ids per 16-byte load
                const uint4 *row = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(ballots) + base);
                for (int32_t t8 = 8 * threadIdx.x; t8 < k; t8 += 8 * 256) {
                    const uint4 v = row[t8 >> 3];
                    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                    for (int e = 0; e < 8; ++e) {
                        const uint32_t raw = (e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xFFFFu);
                        if (t8 + e < k) place(t8 + e, raw == 0xFFFFu ? -1 : (int32_t)raw);
                    }
                }
            } else {
                for (int t = threadIdx.x; t < k; t += 256) place(t, read_id<I32>(ballots, base + t));
            }
        }
        __syncthreads();
        int32_t un0 = 0, un1 = 0;
        auto word = [&](int i) -> uint32_t {
            const int32_t col = c0 + i;
            uint16_t lo = buf[2 * i], hi = buf[2 * i + 1];
            if (col < ncols) {
                un0 += lo == UNSET;
                un1 += hi == UNSET;
            }
            if (FULL) {
                // the candidate a ballot of m-1 entries leaves out is last
                if (col >= m) lo = hi = 0;
                if (lo == UNSET) lo = (uint16_t)(m - 1);
                if (hi == UNSET) hi = has_hi ? (uint16_t)(m - 1) : (uint16_t)0;
            } else {
                // unlisted (and the sentinel column): one shared position
                if (!has_hi) hi = 0;
            }
            return (uint32_t)lo | ((uint32_t)hi << 16);
        };
        if (vec_out) {
            // four words per 16-byte store
            for (int i4 = 4 * threadIdx.x; i4 < cn; i4 += 4 * 256) {
                const uint4 o = make_uint4(word(i4), word(i4 + 1), word(i4 + 2), word(i4 + 3));
                *reinterpret_cast<uint4 *>(pos + q * (int64_t)pitch + c0 + i4) = o;
            }
        } else {
            for (int i = threadIdx.x; i < cn; i += 256) pos[q * (int64_t)pitch + c0 + i] = word(i);
        }
        if (un0) atomicAdd(&unset_cnt[0], un0);
        if (un1) atomicAdd(&unset_cnt[1], un1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int h = 0; h < 2; ++h) {
            if (src[h] < 0) continue;
            if (unset_cnt[h] != ncols - meta.len[src[h]]) set_device_error(err, SCHULZE_EBALLOT);
        }
    }
    }
}

// ------------------------------------------------------------------ position count
// Persistent kernel.  Work units are (tile, chunk of VC voter pairs); each
// workgroup takes a contiguous range of units (equal work per workgroup)
// and flushes its accumulators into acc whenever the tile changes, a
// segment of SEG_PAIRS pairs ends, or its range ends.
//   SQUARE = false: full rankings, tiles X <= Y over candidates; the flush
//                   also writes d[y][x] = voters - d[x][y].
//   SQUARE = true:  truncated ballots over U space, all tiles (X, Y); U
//                   indices map back through ulist; the sentinel column
//                   y = |U| gives R[x].
struct DenseArgs {
    const uint32_t *pos;
    int32_t pitch;  // full rankings: words per position row (multiple of CT)
    int32_t m;
    Meta meta;
    uint32_t *acc;  // m x m
    int64_t lda;
    uint32_t *rsum;
};

__device__ inline void tri_coords(int32_t t, int32_t nb, int32_t &X, int32_t &Y) {
    int32_t x = 0, start = 0;
    while (start + (nb - x) <= t) {
        start += nb - x;
        ++x;
    }
    X = x;
    Y = x + (t - start);
}

template <bool SQUARE>
__global__ __launch_bounds__(CNT_THREADS, 2) void k_count_pos(DenseArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t xs[2][VC][CT];  // two buffers: the chunk counted
    __shared__ __attribute__((aligned(16))) uint32_t ys[2][VC][CT];  // and the next one being staged
    __shared__ uint32_t sred[4][2 * CT];

    if (SQUARE && a.meta.ctr[2] != MODE_DENSE_U) return;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int32_t nvoters = SQUARE ? a.meta.ctr[1] : a.meta.ctr[0];
    const int64_t n_pairs = (nvoters + 1) / 2;
    if (n_pairs == 0) return;
    const int32_t pitch = SQUARE ? a.meta.ctr[4] : a.pitch;
    const int32_t nu = SQUARE ? a.meta.ctr[3] : a.m;
    const int32_t nb = pitch / CT;
    const int64_t ntiles = SQUARE ? (int64_t)nb * nb : (int64_t)nb * (nb + 1) / 2;
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

    auto coords = [&](int32_t t, int32_t &tX, int32_t &tY) {
        if (SQUARE) {
            tX = t / nb;
            tY = t % nb;
        } else {
            tri_coords(t, nb, tX, tY);
        }
    };

    auto load_unit = [&](int64_t u, uint4 (&dst)[8]) {
        const int32_t t = (int32_t)(u / cpt);
        const int64_t chunk = u % cpt;
        int32_t tX, tY;
        coords(t, tX, tY);
        const int32_t col = col4 < 32 ? tX * CT + col4 * 4 : tY * CT + (col4 - 32) * 4;
        const int64_t p0 = chunk * VC;
        for (int q = 0; q < 8; ++q) {
            const int64_t pr = p0 + prow + 4 * q;
            if (pr < n_pairs)
                dst[q] = *reinterpret_cast<const uint4 *>(a.pos + pr * pitch + col);
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
        const int64_t hi = min((int64_t)nvoters, 2 * seg_p1);
        const uint32_t nv = (uint32_t)max((int64_t)0, hi - 2 * seg_p0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int32_t x = X * CT + ty * 8 + i;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t y = Y * CT + tx * 8 + j;
                const uint32_t cnt = (acc[i][j] - sx[i] + sy[j]) >> 16;
                if (SQUARE) {
                    if (x < nu) {
                        const int32_t gx = a.meta.ulist[x];
                        if (y < nu && x != y)
                            atomicAdd(&a.acc[(int64_t)gx * a.lda + a.meta.ulist[y]], cnt);
                        else if (y == nu)
                            atomicAdd(&a.rsum[gx], cnt);
                    }
                } else if (x < nu && y < nu && x != y) {
                    atomicAdd(&a.acc[(int64_t)x * a.lda + y], cnt);
                    if (X != Y) atomicAdd(&a.acc[(int64_t)y * a.lda + x], nv - cnt);
                }
                acc[i][j] = 0u;
            }
        }
        for (int e = 0; e < 4; ++e) s4[e] = 0u;
    };

    const us2 ones = {1, 1};
    // staged words into LDS buffer sb, their column sums added to sadd
    auto stage_write = [&](int sb, uint32_t (&sadd)[4]) {
        for (int q = 0; q < 8; ++q) {
            const int pr = prow + 4 * q;
            uint32_t *dst = col4 < 32 ? &xs[sb][pr][col4 * 4] : &ys[sb][pr][(col4 - 32) * 4];
            *reinterpret_cast<uint4 *>(dst) = stage[q];
            sadd[0] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, stage[q].x), ones, sadd[0], false);
            sadd[1] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, stage[q].y), ones, sadd[1], false);
            sadd[2] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, stage[q].z), ones, sadd[2], false);
            sadd[3] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, stage[q].w), ones, sadd[3], false);
        }
    };

    // Unit u is counted from one LDS buffer while unit u+1 is staged into the
    // other: one barrier per unit.  The next unit's column sums wait in s4n
    // until the current segment has been flushed.
    load_unit(u0, stage);
    stage_write(0, s4);
    __syncthreads();
    int cur = 0;
    for (int64_t u = u0; u < u1; ++u) {
        const int32_t t = (int32_t)(u / cpt);
        const int64_t chunk = u % cpt;
        if (t != cur_tile) {
            cur_tile = t;
            coords(t, X, Y);
            seg_p0 = chunk * VC;
        } else if (chunk % SEGC == 0) {
            seg_p0 = chunk * VC;
        }
        seg_p1 = min(n_pairs, (chunk + 1) * VC);
        const bool more = u + 1 < u1;
        if (more) load_unit(u + 1, stage);  // overlaps the compute below

        // Two voter pairs per iteration, the LDS reads of each pair issued
        // before the products of the previous one (scheduling barriers keep
        // them there), so that their latency hides behind 128 VALU
        // instructions.
        const uint32_t(*xb)[CT] = cur ? xs[1] : xs[0];  // (selects: no dynamically indexed arrays)
        const uint32_t(*yb)[CT] = cur ? ys[1] : ys[0];
        auto read_pair = [&](int v, uint4 (&q)[4]) {
            q[0] = *reinterpret_cast<const uint4 *>(&xb[v][ty * 8]);
            q[1] = *reinterpret_cast<const uint4 *>(&xb[v][ty * 8 + 4]);
            q[2] = *reinterpret_cast<const uint4 *>(&yb[v][tx * 8]);
            q[3] = *reinterpret_cast<const uint4 *>(&yb[v][tx * 8 + 4]);
        };
        auto count_pair = [&](const uint4 (&q)[4]) {
            const uint32_t xv[8] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w};
            const uint32_t yv[8] = {q[2].x, q[2].y, q[2].z, q[2].w, q[3].x, q[3].y, q[3].z, q[3].w};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const us2 xi = __builtin_bit_cast(us2, xv[i]);
                us2 diff[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) diff[j] = xi - __builtin_bit_cast(us2, yv[j]);
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_udot2(diff[j], ones, acc[i][j], false);
            }
        };
        static_assert(VC % 2 == 0 && (VC & (VC - 1)) == 0, "voter pairs per chunk");
        uint4 qa[4], qb[4];
        read_pair(0, qa);
#pragma unroll 1
        for (int v = 0; v < VC; v += 2) {
            read_pair(v + 1, qb);
            __builtin_amdgcn_sched_barrier(0);
            count_pair(qa);
            read_pair((v + 2) & (VC - 1), qa);  // (after the last pair: pair 0 again, unused)
            __builtin_amdgcn_sched_barrier(0);
            count_pair(qb);
        }
        uint32_t s4n[4] = {0u, 0u, 0u, 0u};
        if (more) stage_write(cur ^ 1, s4n);
        __syncthreads();  // the next unit is staged; everyone is done with this one

        bool boundary = !more;
        if (more) {
            const int32_t tn = (int32_t)((u + 1) / cpt);
            const int64_t cn = (u + 1) % cpt;
            boundary = tn != t || cn % SEGC == 0;
        }
        if (boundary) flush();
        for (int e = 0; e < 4; ++e) s4[e] += s4n[e];
        cur ^= 1;
    }
}

// ------------------------------------------------------------------ pair scattering
// One wavefront per truncated ballot: lane t handles listed entry t.  For
// every earlier entry i < t the pair (c_i before c_t) adds the voter's
// weight to C[c_i][c_t], i.e. subtracts it from acc[c_t][c_i]; every listed
// entry adds the weight to R.  Equal entries are a repeated id.
template <bool I32>
__global__ __launch_bounds__(256) void k_count_pairs(const void *__restrict__ ballots, int32_t L,
                                                     int32_t m, const uint32_t *__restrict__ weight, Meta meta,
                                                     uint32_t *__restrict__ acc, int64_t lda,
                                                     uint32_t *__restrict__ rsum, int32_t *err) {
    if (meta.ctr[2] != MODE_SPARSE) return;
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (slot >= meta.ctr[1]) return;
    const int32_t v = meta.trunc_src[slot];
    const int32_t k = meta.len[v];
    const uint32_t w = weight ? weight[v] : 1u;
    const int64_t base = (int64_t)v * L;
    bool dup = false;
    for (int t = lane; t < k; t += 64) {
        const int32_t ct = read_id<I32>(ballots, base + t);
        if (ct < 0 || ct >= m) continue;  // reported by the scan
        if (w) atomicAdd(&rsum[ct], w);
        uint32_t *row = acc + (int64_t)ct * lda;
        for (int i = 0; i < t; ++i) {
            const int32_t ci = read_id<I32>(ballots, base + i);
            if (ci == ct) dup = true;
            if (w && ci >= 0 && ci < m) atomicSub(&row[ci], w);
        }
    }
    if (__ballot(dup) && lane == 0) set_device_error(err, SCHULZE_EBALLOT);
}

// ------------------------------------------------------------------ bucketed pair counting
// The same sums as k_count_pairs without its random device-wide atomics into
// the m x m accumulator.  The listed entries ("occurrences") of truncated
// ballots are bucketed by candidate (a counting sort: per-workgroup
// histograms in LDS over fixed ballot ranges, column prefixes, placement),
// and then each candidate r's row of C^T (C[y][r] = weight of ballots
// listing y before r) is accumulated in LDS from the ballot prefixes ahead
// of its occurrences; d[r][y] = R_r - C[y][r] (plus any full-ranking
// counts).  A candidate with at most OCC_CHUNK occurrences is one work item
// that writes its row of d at once; a heavier one is split into items that
// write their partial rows to a buffer, summed by the finish.  Nothing here
// needs the m x m accumulator unless full rankings are counted as well.
constexpr int OCC_CHUNK = 8192;            // occurrences per accumulation item (<= 65535: packed counts)
constexpr int32_t OCC_MAX_M = 32768;       // an LDS row of counts
constexpr int64_t OCC_MAX = (int64_t)1 << 27;  // occurrence buffer limit (entries)
constexpr int OCC_FIN_COLS = 2048;         // columns per unit of the finish
constexpr int FIN_COUNT = 5;               // meta.ctr slot: rows listed for the finish

struct OccArgs {
    const void *ballots;
    int dtype32;
    int32_t L, m;
    int64_t n;
    int32_t tbits;        // occurrence word: ballot << tbits | position
    int32_t row_vec;      // uint16 ids, even L, 4-byte aligned rows: rows read as 32-bit words (1), or as
                          // 16-byte pieces (2: the ballots 16-byte aligned and n L ids whole pieces)
    const uint32_t *weight;
    Meta meta;
    uint32_t *hist;       // G x m: per-workgroup counts, then their exclusive prefix over workgroups
    uint32_t *row_start;  // m + 1: occurrences per candidate, then the exclusive scan
    uint32_t *item_start; // m + 1: accumulation items per candidate, then the exclusive scan
    uint32_t *part_start; // m + 1: partial rows per candidate (its items if more than one), then the scan
    int32_t *fin;         // candidates whose rows the finish writes (no occurrences, or two or more items);
                          // their number in meta.ctr[FIN_COUNT]
    uint32_t *occ;        // placed occurrences
    void *partial;        // partial rows, pitch ppitch elements (uint16 for unit weights, else uint32)
    int64_t ppitch;
    uint32_t *acc;
    int64_t lda;
    uint32_t *rsum;
    int32_t *err;
};

// Eight consecutive values of a row of d: 16-byte stores when the row is
// aligned for them and all eight columns exist, else one at a time.
template <typename T>
__device__ inline void store8(T *__restrict__ drow, int32_t y, int32_t m, bool vec, const uint32_t (&v)[8]) {
    if (vec && y + 8 <= m) {
        if constexpr (sizeof(T) == 4) {
            reinterpret_cast<uint4 *>(drow + y)[0] = make_uint4(v[0], v[1], v[2], v[3]);
            reinterpret_cast<uint4 *>(drow + y)[1] = make_uint4(v[4], v[5], v[6], v[7]);
        } else {
            reinterpret_cast<uint4 *>(drow + y)[0] =
                make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
        }
        return;
    }
    for (int u = 0; u < 8 && y + u < m; ++u) drow[y + u] = (T)v[u];
}

// Ballots of bucketing workgroup g: [v0, v1) (the same in both passes).
__device__ inline void occ_range(int64_t n, int64_t &v0, int64_t &v1) {
    v0 = n * blockIdx.x / gridDim.x;
    v1 = n * (blockIdx.x + 1) / gridDim.x;
}

// PLACE = false: hist[g][c] = occurrences of c in workgroup g's ballots.
// PLACE = true:  write them to occ[] at row_start[c] + hist[g][c] + k.
// Rows of L <= 64 entries: a wavefront takes 64 / L ballots at once, one
// lane per entry; a ballot ends at its first padding entry (a wavefront
// ballot of the padding lanes gives it), and full rankings (m - 1 or more
// listed) are left to the dense count.  Longer rows: one ballot per
// wavefront, 64 entries at a time.
template <int MAXM, bool PLACE, bool I32>
__global__ __launch_bounds__(256) void k_occ_bucket(OccArgs a) {
    __shared__ uint32_t cnt[MAXM];
    if (a.meta.ctr[2] != MODE_SPARSE) return;
    const int32_t m = a.m, L = a.L;
    const int64_t hrow = (int64_t)blockIdx.x * m;
    if (PLACE) {
        // the workgroup's first slot per candidate, PRO candidates per thread
        // with every load in flight at once (one at a time, the loads took
        // most of the pass)
        constexpr int PRO = 16;
        for (int32_t c0 = threadIdx.x; c0 < m; c0 += 256 * PRO) {
            uint32_t rs[PRO], hs[PRO];
            for (int u = 0; u < PRO; ++u) {
                const int32_t c = c0 + 256 * u < m ? c0 + 256 * u : 0;
                rs[u] = a.row_start[c];
                hs[u] = a.hist[hrow + c];
            }
            for (int u = 0; u < PRO; ++u)
                if (c0 + 256 * u < m) cnt[c0 + 256 * u] = rs[u] + hs[u];
        }
    } else {
        for (int32_t c = threadIdx.x; c < m; c += 256) cnt[c] = 0u;
    }
    __syncthreads();
    int64_t v0, v1;
    occ_range(a.n, v0, v1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto put = [&](int64_t v, int32_t t, int32_t c) {
        const uint32_t q = atomicAdd(&cnt[c], 1u);
        if (PLACE) a.occ[q] = ((uint32_t)v << a.tbits) | (uint32_t)t;
    };
    if (L <= 64) {
        const int32_t bpw = 64 / L;  // ballots per wavefront step
        const int32_t sub = lane / L, t = lane - sub * L;
        const bool lane_ok = sub < bpw;
        const uint64_t lane_bits = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
        constexpr int U = 4;  // steps in flight
        for (int64_t vb = v0 + (int64_t)wave * bpw; vb < v1; vb += (int64_t)4 * bpw * U) {
            int32_t c[U];
            int64_t vv[U];
            for (int u = 0; u < U; ++u) {
                vv[u] = vb + (int64_t)4 * bpw * u + sub;
                // (every lane loads: a load under a condition is waited for inside it)
                c[u] = (int32_t)load_raw<I32>(a.ballots, lane_ok && vv[u] < v1 ? vv[u] * L + t : 0);
            }
            for (int u = 0; u < U; ++u) c[u] = lane_ok && vv[u] < v1 ? raw_id<I32>((uint32_t)c[u]) : -2;
            for (int u = 0; u < U; ++u) {
                const uint64_t pad = __ballot(c[u] < 0);  // -1 padding, -2 no ballot
                const uint64_t mine = lane_ok ? (pad >> (sub * L)) & lane_bits : lane_bits;
                const int32_t k = mine ? (int32_t)__builtin_ctzll(mine) : L;
                if (c[u] >= 0 && c[u] < m && t < k && k < m - 1) put(vv[u], t, c[u]);
            }
        }
    } else {
        for (int64_t v = v0 + wave; v < v1; v += 4) {
            const int32_t k = a.meta.len[v];
            if (k >= m - 1) continue;
            for (int32_t t = lane; t < k; t += 64) {
                const int32_t c = read_id<I32>(a.ballots, v * L + t);
                if (c >= 0 && c < m) put(v, t, c);
            }
        }
    }
    if (!PLACE) {
        __syncthreads();
        for (int32_t c = threadIdx.x; c < m; c += 256) a.hist[hrow + c] = cnt[c];
    }
}

// 64 candidates per workgroup, the G histogram rows split over COL_GROUPS
// thread groups (enough loads in flight to stream the histograms):
// hist[g][c] becomes its exclusive prefix over g; per candidate c,
// row_start[c] = occurrences, item_start[c] = accumulation items,
// part_start[c] = partial rows (its items when there are two or more), and
// the candidates whose rows the finish writes are listed.
constexpr int COL_GROUPS = 16;
__global__ __launch_bounds__(64 * COL_GROUPS) void k_occ_columns(OccArgs a, int32_t G) {
    __shared__ uint32_t part[COL_GROUPS][64];
    if (a.meta.ctr[2] != MODE_SPARSE) return;
    const int32_t c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int grp = threadIdx.x >> 6;
    const int32_t g0 = G * grp / COL_GROUPS, g1 = G * (grp + 1) / COL_GROUPS;
    uint32_t sum = 0;
    if (c < a.m)
        for (int32_t g = g0; g < g1; ++g) sum += a.hist[(int64_t)g * a.m + c];
    part[grp][threadIdx.x & 63] = sum;
    __syncthreads();
    if (c >= a.m) return;
    uint32_t run = 0;
    for (int q = 0; q < grp; ++q) run += part[q][threadIdx.x & 63];
    for (int32_t g = g0; g < g1; ++g) {
        const uint32_t h = a.hist[(int64_t)g * a.m + c];
        a.hist[(int64_t)g * a.m + c] = run;
        run += h;
    }
    if (grp == COL_GROUPS - 1) {
        const uint32_t items = (run + OCC_CHUNK - 1) / OCC_CHUNK;
        a.row_start[c] = run;
        a.item_start[c] = items;
        a.part_start[c] = items > 1 ? items : 0u;
        if (items != 1) a.fin[atomicAdd(&a.meta.ctr[FIN_COUNT], 1)] = c;
    }
}

// One workgroup of 1024 threads: exclusive scans of the three per-candidate
// counts, totals at [m].  A thread takes `per` consecutive candidates, read
// and written as 16-byte vectors when per is a multiple of 4 (at most
// SCAN_VEC of them per array in registers), else one at a time.
constexpr int SCAN_VEC = 8;
__global__ __launch_bounds__(1024) void k_occ_scan(OccArgs a) {
    __shared__ uint32_t part[3][1024];
    if (a.meta.ctr[2] != MODE_SPARSE) return;
    const int32_t m = a.m;
    const int32_t per = (m + 1023) / 1024;
    const int32_t c0 = min(m, (int32_t)threadIdx.x * per), c1 = min(m, c0 + per);
    uint32_t *arr[3] = {a.row_start, a.item_start, a.part_start};
    uint32_t s[3] = {0u, 0u, 0u};
    const bool vec = per % 4 == 0 && per / 4 <= SCAN_VEC && c1 - c0 == per;
    uint4 v[3][SCAN_VEC];
    if (vec) {
        for (int q = 0; q < 3; ++q)
            for (int k = 0; k < SCAN_VEC; ++k)
                if (k < per / 4) v[q][k] = reinterpret_cast<const uint4 *>(arr[q] + c0)[k];
        for (int q = 0; q < 3; ++q)
            for (int k = 0; k < SCAN_VEC; ++k)
                if (k < per / 4) s[q] += v[q][k].x + v[q][k].y + v[q][k].z + v[q][k].w;
    } else {
        for (int q = 0; q < 3; ++q)
            for (int32_t c = c0; c < c1; ++c) s[q] += arr[q][c];
    }
    for (int q = 0; q < 3; ++q) part[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t add[3];
        for (int q = 0; q < 3; ++q) add[q] = (int)threadIdx.x >= off ? part[q][threadIdx.x - off] : 0u;
        __syncthreads();
        for (int q = 0; q < 3; ++q) part[q][threadIdx.x] += add[q];
        __syncthreads();
    }
    for (int q = 0; q < 3; ++q) {
        uint32_t run = part[q][threadIdx.x] - s[q];
        if (vec) {
            for (int k = 0; k < SCAN_VEC; ++k) {
                if (k >= per / 4) break;
                uint4 o;
                o.x = run, run += v[q][k].x;
                o.y = run, run += v[q][k].y;
                o.z = run, run += v[q][k].z;
                o.w = run, run += v[q][k].w;
                reinterpret_cast<uint4 *>(arr[q] + c0)[k] = o;
            }
        } else {
            for (int32_t c = c0; c < c1; ++c) {
                const uint32_t x = arr[q][c];
                arr[q][c] = run;
                run += x;
            }
        }
        if (threadIdx.x == 1023) arr[q][m] = part[q][1023];
    }
}

// Accumulation item `blockIdx.x`: a chunk of one candidate r's occurrences.
// For an occurrence of r at position t of ballot v, every id ahead of it
// gains the voter's weight in the LDS row (C[id][r]), and r gains it in R.
// PACKED (unit weights): two 16-bit counts per LDS word (an item adds at
// most OCC_CHUNK to a column).  A thread takes its occurrences B at a time
// and, for rows read as 32-bit words, issues every row load of the batch
// before the first LDS update, so that many loads are in flight.  The only
// item of a row writes the row of d (d[r][y] = base + R - C[y][r], base =
// full-ranking counts in acc or 0); an item of a heavier row writes its
// counts to its partial row and adds its part of R to rsum[r].
template <int MAXM, bool PACKED, typename T, int WMAX, bool PIECES, bool I32>
__global__ __launch_bounds__(256) void k_occ_accumulate(OccArgs a, T *__restrict__ d, int64_t ldd, uint32_t limit,
                                                        uint8_t *__restrict__ over_flag, int acc_zero, int dvec) {
    constexpr int WORDS = PACKED ? MAXM / 2 : MAXM;
    constexpr int B = WMAX <= 16 ? 2 : 1;  // occurrences per batch
    __shared__ __attribute__((aligned(16))) uint32_t row[WORDS];
    __shared__ uint32_t wsum;
    __shared__ int32_t sh_r, sh_nitems, sh_k;
    __shared__ uint32_t sh_b, sh_e;
    if (a.meta.ctr[2] != MODE_SPARSE) return;
    const int32_t m = a.m;
    const uint32_t item = blockIdx.x;
    if (item >= a.item_start[m]) return;
    if (threadIdx.x == 0) {
        // the candidate whose item range holds `item` (binary search)
        int32_t lo = 0, hi = m - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (a.item_start[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const uint32_t k = item - a.item_start[lo];
        const uint32_t b = a.row_start[lo] + k * OCC_CHUNK;
        sh_r = lo;
        sh_k = (int32_t)k;
        sh_nitems = (int32_t)(a.item_start[lo + 1] - a.item_start[lo]);
        sh_b = b;
        sh_e = min(a.row_start[lo + 1], b + (uint32_t)OCC_CHUNK);
        wsum = 0;
    }
    const int32_t words = PACKED ? (m + 1) / 2 : m;
    const int32_t words4 = (words + 3) / 4;
    uint4 *row4 = reinterpret_cast<uint4 *>(row);
    for (int32_t c = threadIdx.x; c < words4; c += 256) row4[c] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const int32_t r = sh_r;
    const uint32_t tmask = (1u << a.tbits) - 1u;
    uint32_t wpart = 0;
    bool dup = false;
    auto add = [&](int32_t id, uint32_t w) {
        if (id == r) dup = true;
        if (id < 0 || id >= m) return;
        if (PACKED)
            atomicAdd(&row[id >> 1], 1u << ((id & 1) * 16));
        else
            atomicAdd(&row[id], w);
    };
    constexpr int WN = WMAX > 0 ? WMAX : 1;
    if (WMAX > 0 && PIECES) {
        // uint16 ids, rows of even length, ballots 16-byte aligned and a
        // whole number of 16-byte pieces: a row's words (two ids each) are
        // read as the 16-byte pieces that hold them.  A scattered load costs
        // the load path about a cycle per lane whatever its width, so an
        // occurrence takes about two wide loads instead of one per word.
        constexpr int NCH = (WMAX + 3) / 4 + 1;  // pieces that hold WMAX words at any offset
        const uint32_t *words32 = static_cast<const uint32_t *>(a.ballots);
        const int64_t wrow = a.L / 2;
        constexpr int PB = 2;  // occurrences per thread in flight
        for (uint32_t q0 = sh_b + threadIdx.x; q0 < sh_e; q0 += 256 * PB) {
            uint32_t ov[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) ov[u] = q0 + 256 * u < sh_e ? a.occ[q0 + 256 * u] : 0u;
            uint32_t f[PB][4 * NCH];
            int32_t tt[PB], sk[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int64_t v = ov[u] >> a.tbits;
                tt[u] = q0 + 256 * u < sh_e ? (int32_t)(ov[u] & tmask) : 0;
                const int32_t nw = (tt[u] + 1) / 2;
                const uint32_t *rw = words32 + v * wrow;
                sk[u] = (int32_t)((reinterpret_cast<uintptr_t>(rw) >> 2) & 3);  // words before the row
                const uint4 *rc = reinterpret_cast<const uint4 *>(rw - sk[u]);
                const int32_t nch = (sk[u] + nw + 3) >> 2;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    uint4 x = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
                    if (c < nch) x = rc[c];
                    f[u][4 * c] = x.x, f[u][4 * c + 1] = x.y, f[u][4 * c + 2] = x.z, f[u][4 * c + 3] = x.w;
                }
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const bool ok = q0 + 256 * u < sh_e;
                const uint32_t w = !ok ? 0u : (PACKED ? 1u : (a.weight ? a.weight[ov[u] >> a.tbits] : 1u));
                wpart += w;
                // word j of the row to f[u][j]: shifts by one and by two words
                // under masks (opaque to the compiler, which would otherwise
                // index the array by the offset and move it to scratch memory)
                uint32_t m1 = (sk[u] & 1) ? 0xFFFFFFFFu : 0u, m2 = (sk[u] & 2) ? 0xFFFFFFFFu : 0u;
                asm volatile("" : "+v"(m1), "+v"(m2));
#pragma unroll
                for (int j = 0; j + 1 < 4 * NCH; ++j) f[u][j] = (f[u][j] & ~m1) | (f[u][j + 1] & m1);
#pragma unroll
                for (int j = 0; j + 2 < 4 * NCH; ++j) f[u][j] = (f[u][j] & ~m2) | (f[u][j + 2] & m2);
#pragma unroll
                for (int j = 0; j < WMAX; ++j) {
                    if (2 * j < tt[u] && w != 0) {
                        add((int32_t)(f[u][j] & 0xFFFFu), w);
                        if (2 * j + 1 < tt[u]) add((int32_t)(f[u][j] >> 16), w);
                    }
                }
            }
        }
    } else if (WMAX > 0 && a.row_vec) {
        // uint16 ids, rows of even length read as 32-bit words (two ids each)
        const uint32_t *words32 = static_cast<const uint32_t *>(a.ballots);
        const int64_t wrow = a.L / 2;
        for (uint32_t q0 = sh_b + threadIdx.x; q0 < sh_e; q0 += 256 * B) {
            uint32_t ov[B];
            for (int u = 0; u < B; ++u) ov[u] = q0 + 256 * u < sh_e ? a.occ[q0 + 256 * u] : 0u;
            uint32_t wd[B][WN];
            int32_t tt[B];
            uint32_t ww[B];
            for (int u = 0; u < B; ++u) {
                const bool ok = q0 + 256 * u < sh_e;
                const int64_t v = ov[u] >> a.tbits;
                tt[u] = ok ? (int32_t)(ov[u] & tmask) : 0;
                ww[u] = ok ? (PACKED ? 1u : (a.weight ? a.weight[v] : 1u)) : 0u;
                const int32_t nw = (tt[u] + 1) / 2;
                const uint32_t *rw = words32 + v * wrow;
                for (int j = 0; j < WN; ++j) wd[u][j] = j < nw ? rw[j] : 0xFFFFFFFFu;
            }
            for (int u = 0; u < B; ++u) {
                wpart += ww[u];
                if (ww[u] == 0) continue;
                for (int j = 0; j < WN; ++j) {
                    if (2 * j >= tt[u]) break;
                    const uint32_t x = wd[u][j];
                    add((int32_t)(x & 0xFFFFu), ww[u]);
                    if (2 * j + 1 < tt[u]) add((int32_t)(x >> 16), ww[u]);
                }
            }
        }
    } else {
        for (uint32_t q = sh_b + threadIdx.x; q < sh_e; q += 256) {
            const uint32_t ovq = a.occ[q];
            const int64_t v = ovq >> a.tbits;
            const int32_t t = (int32_t)(ovq & tmask);
            const uint32_t w = PACKED ? 1u : (a.weight ? a.weight[v] : 1u);
            wpart += w;
            if (w == 0) continue;
            const int64_t base = v * a.L;
            // sixteen ids in flight, every load unconditional (positions past t
            // repeat the last one and are not added)
            for (int32_t i0 = 0; i0 < t; i0 += 16) {
                uint32_t raw[16];
                for (int u = 0; u < 16; ++u) raw[u] = load_raw<I32>(a.ballots, base + min(i0 + u, t - 1));
                for (int u = 0; u < 16; ++u)
                    if (i0 + u < t) add(raw_id<I32>(raw[u]), w);
            }
        }
    }
    if (wpart) atomicAdd(&wsum, wpart);
    if (__ballot(dup) && (threadIdx.x & 63) == 0) set_device_error(a.err, SCHULZE_EBALLOT);
    __syncthreads();
    if (sh_nitems == 1) {
        // the row's only item: d[r][y] = base + R - C[y][r]; the finish skips the row
        const uint32_t R = wsum;
        const uint32_t *arow = a.acc + (int64_t)r * a.lda;
        bool over = false;
        T *drow = d + (int64_t)r * ldd;
        for (int32_t y = 8 * threadIdx.x; y < m; y += 8 * 256) {  // eight columns per thread and step
            uint32_t v[8];
            for (int e = 0; e < 8; ++e) {
                const int32_t yy = y + e;
                v[e] = 0u;
                if (yy >= m || yy == r) continue;
                const uint32_t cnt = PACKED ? (row[yy >> 1] >> ((yy & 1) * 16)) & 0xFFFFu : row[yy];
                v[e] = (acc_zero ? 0u : arow[yy]) - cnt + R;
                if (v[e] > limit) {
                    over = true;
                    v[e] = limit;
                }
            }
            store8<T>(drow, y, m, dvec != 0, v);
        }
        // reported by the finish, after every ballot error of this launch
        if (over) over_flag[0] = 1;
        return;
    }
    // an item of a heavier row: its partial row (same element layout as the LDS row)
    uint4 *prow = reinterpret_cast<uint4 *>(static_cast<uint32_t *>(a.partial) +
                                            (int64_t)(a.part_start[r] + sh_k) * (a.ppitch * (PACKED ? 1 : 2) / 2));
    for (int32_t c = threadIdx.x; c < words4; c += 256) prow[c] = row4[c];
    if (threadIdx.x == 0 && wsum) atomicAdd(&a.rsum[r], wsum);
}

// Rows the accumulation items did not finish: candidates without
// occurrences (d[r][y] = base) and heavier candidates (d[r][y] = base + R_r
// - sum of their partial rows), as listed by the column pass.  Persistent:
// units (listed row, block of OCC_FIN_COLS columns) dealt to the
// workgroups in turn (a walk over every row that skipped the finished ones
// waited for memory at each); a thread takes eight consecutive columns (one
// 16-byte read per partial row of unit weights), four partial rows in
// flight.  Also reports an overflow found by the accumulation.
template <typename T, bool PACKED>
__global__ __launch_bounds__(256) void k_occ_finish(OccArgs a, T *__restrict__ d, int64_t ldd, uint32_t limit,
                                                    const uint8_t *__restrict__ over_flag, int acc_zero, int dvec) {
    static_assert(OCC_FIN_COLS == 8 * 256, "a thread takes eight columns");
    if (a.meta.ctr[2] != MODE_SPARSE) return;
    const int32_t m = a.m;
    if (blockIdx.x == 0 && threadIdx.x == 0 && over_flag[0]) set_device_error(a.err, SCHULZE_ERANGE);
    const int32_t cb = (m + OCC_FIN_COLS - 1) / OCC_FIN_COLS;
    const bool avec = (a.lda % 4) == 0;  // rows of acc 16-byte aligned
    const int32_t nfin = a.meta.ctr[FIN_COUNT];
    bool over = false;
    for (int64_t u = blockIdx.x; u < (int64_t)nfin * cb; u += gridDim.x) {
        const int32_t r = a.fin[u / cb];
        const int32_t y = (int32_t)(u % cb) * OCC_FIN_COLS + 8 * threadIdx.x;
        if (y >= m) continue;
        const uint32_t p0 = a.part_start[r], np = a.part_start[r + 1] - p0;
        const uint32_t R = np ? a.rsum[r] : 0u;
        uint32_t c[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        // partial rows hold round_up(m, 8) columns: eight at y are always there
        auto add_row = [&](uint32_t k) {
            const int64_t off = (int64_t)(p0 + k) * a.ppitch + y;
            if constexpr (PACKED) {
                const uint4 x = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(a.partial) + off);
                const uint32_t w[4] = {x.x, x.y, x.z, x.w};
                for (int e = 0; e < 4; ++e) {
                    c[2 * e] += w[e] & 0xFFFFu;
                    c[2 * e + 1] += w[e] >> 16;
                }
            } else {
                const uint4 *q = reinterpret_cast<const uint4 *>(static_cast<const uint32_t *>(a.partial) + off);
                const uint4 x0 = q[0], x1 = q[1];
                c[0] += x0.x, c[1] += x0.y, c[2] += x0.z, c[3] += x0.w;
                c[4] += x1.x, c[5] += x1.y, c[6] += x1.z, c[7] += x1.w;
            }
        };
        uint32_t k = 0;
        for (; k + 4 <= np; k += 4) {
            add_row(k);
            add_row(k + 1);
            add_row(k + 2);
            add_row(k + 3);
        }
        for (; k < np; ++k) add_row(k);
        uint32_t base[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        if (!acc_zero) {
            const uint32_t *arow = a.acc + (int64_t)r * a.lda;
            if (avec && y + 8 <= m) {
                const uint4 b0 = *reinterpret_cast<const uint4 *>(arow + y), b1 = *reinterpret_cast<const uint4 *>(arow + y + 4);
                base[0] = b0.x, base[1] = b0.y, base[2] = b0.z, base[3] = b0.w;
                base[4] = b1.x, base[5] = b1.y, base[6] = b1.z, base[7] = b1.w;
            } else {
                for (int e = 0; e < 8 && y + e < m; ++e) base[e] = arow[y + e];
            }
        }
        uint32_t v[8];
        for (int e = 0; e < 8; ++e) {
            v[e] = y + e == r ? 0u : base[e] - c[e] + R;
            if (v[e] > limit) {
                over = true;
                v[e] = limit;
            }
        }
        store8<T>(d + (int64_t)r * ldd, y, m, dvec != 0, v);
    }
    if (over) set_device_error(a.err, SCHULZE_ERANGE);
}

// ------------------------------------------------------------------ weighted full rankings
// Full rankings with voter weights: plain compare-and-add per voter (the
// modular trick needs unit weights to bound a segment's total).
__global__ __launch_bounds__(256) void k_count_full_weighted(const uint32_t *__restrict__ weight, Meta meta,
                                                             const uint32_t *__restrict__ pos, int32_t pitch, int32_t m,
                                                             uint32_t *__restrict__ acc, int64_t lda) {
    // one thread per (x, y) pair of a 16 x 16 block, looping over voters
    const int32_t x = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int32_t y = blockIdx.x * 16 + (threadIdx.x & 15);
    const int32_t n_full = meta.ctr[0];
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
// d[x][y] = acc[x][y] plus the truncated ballots' R term, 0 on the
// diagonal; range-checked store.
template <typename T>
__global__ __launch_bounds__(256) void k_count_finish(const uint32_t *__restrict__ acc, int64_t lda,
                                                      const uint32_t *__restrict__ rsum, Meta meta, int32_t m,
                                                      T *__restrict__ d, int64_t ldd, uint32_t limit, int32_t *err,
                                                      int bucketed) {
    // one workgroup per row x; the bucketed route writes its own rows
    const int32_t x = blockIdx.x;
    if (bucketed && meta.ctr[2] == MODE_SPARSE) return;
    const bool dense_u = meta.ctr[2] == MODE_DENSE_U;
    const uint32_t rx = rsum[x];
    const bool in_x = dense_u && meta.in_u[x];
    bool over = false;
    for (int32_t y = threadIdx.x; y < m; y += 256) {
        uint32_t v = 0u;
        if (x != y) {
            v = acc[(int64_t)x * lda + y];
            // pair scattering: acc holds -C^T, add R[x]; dense over U: U x U is
            // complete, x in U beats every y outside U on the R[x] ballots
            if (!dense_u || (in_x && !meta.in_u[y])) v += rx;
        }
        if (v > limit) {
            over = true;
            v = limit;
        }
        d[(int64_t)x * ldd + y] = (T)v;
    }
    if (over) set_device_error(err, SCHULZE_ERANGE);
}

// Byte layout of WS_BALLOT_META for n ballots and m candidates.
// Total voter weight in 64 bits: counts accumulate in 32-bit words, which
// cannot wrap while the total stays below 2^32 (and then the finish checks
// every count against the value type); a total of 2^32 or more sets
// SCHULZE_ERANGE.  total and done start at zero; the last workgroup to add
// its part decides.
__global__ __launch_bounds__(256) void k_weight_total(const uint32_t *__restrict__ w, int64_t n,
                                                      unsigned long long *total, int32_t *done, int32_t *err) {
    __shared__ unsigned long long part[256];
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += w[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(total, part[0]);
        __threadfence();
        if (atomicAdd(done, 1) == (int32_t)gridDim.x - 1) {
            __threadfence();
            if (atomicAdd(total, 0ull) >> 32) set_device_error(err, SCHULZE_ERANGE);
        }
    }
}

// Zero the m x m accumulator, unless skip_bucketed and the device chose the
// bucketed route (which then does not read it).
__global__ __launch_bounds__(256) void k_fill_acc(uint32_t *__restrict__ p, int64_t words, Meta meta,
                                                  int skip_bucketed) {
    if (skip_bucketed && meta.ctr[2] == MODE_SPARSE) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);  // workspace: 16-byte aligned
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t j = i; j < words / 4; j += stride) p4[j] = z;
    for (int64_t j = words / 4 * 4 + i; j < words; j += stride) p[j] = 0u;
}

struct MetaLayout {
    size_t ctr, k2, len, full_src, trunc_src, in_u, ulist, umap, total;
    MetaLayout(int64_t n, int32_t m) {
        size_t o = 0;
        auto take = [&](size_t bytes) {
            size_t at = o;
            o += (bytes + 255) / 256 * 256;
            return at;
        };
        ctr = take(64 * sizeof(int32_t));
        k2 = take(NPART * sizeof(unsigned long long));
        len = take(sizeof(int32_t) * (size_t)n);
        full_src = take(sizeof(int32_t) * (size_t)n);
        trunc_src = take(sizeof(int32_t) * (size_t)n);
        in_u = take((size_t)m);
        ulist = take(sizeof(int32_t) * (size_t)m);
        umap = take(sizeof(int32_t) * (size_t)m);
        total = o;
    }
};

// Byte layout of WS_OCC for G bucketing workgroups, m candidates and at
// most cap occurrences.
// Partial rows: every item of a candidate with two or more items has one,
// and such a candidate has more than OCC_CHUNK occurrences, so there are at
// most 2 cap / OCC_CHUNK of them.
struct OccLayout {
    size_t hist, row_start, item_start, part_start, fin, occ, partial, over_flag, total;
    int64_t ppitch, max_parts;
    OccLayout(int64_t G, int32_t m, int64_t cap, size_t partial_elem) {
        size_t o = 0;
        auto take = [&](size_t bytes) {
            size_t at = o;
            o += (bytes + 255) / 256 * 256;
            return at;
        };
        ppitch = round_up(m, 8);
        max_parts = cap > 0 ? 2 * ceil_div(cap, OCC_CHUNK) + 1 : 0;
        hist = take(sizeof(uint32_t) * (size_t)G * m);
        row_start = take(sizeof(uint32_t) * ((size_t)m + 1));
        item_start = take(sizeof(uint32_t) * ((size_t)m + 1));
        part_start = take(sizeof(uint32_t) * ((size_t)m + 1));
        occ = take(sizeof(uint32_t) * (size_t)cap);
        partial = take(partial_elem * (size_t)max_parts * (size_t)ppitch);
        fin = take(sizeof(int32_t) * (size_t)m);
        over_flag = take(sizeof(uint32_t));  // a count above the limit was clamped
        total = o;
    }
};

// The counting (PLACE = false) or placing pass of the bucketing, for the LDS
// histogram that fits m and the ballots' id type.
template <bool PLACE>
int occ_bucket(schulze_ctx *ctx, hipStream_t s, const OccArgs &oa, dim3 g) {
    const dim3 b(256);
    if (oa.m <= OCC_MAX_M / 2) {
        if (oa.dtype32)
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s, (k_occ_bucket<OCC_MAX_M / 2, PLACE, true><<<g, b, 0, s>>>(oa)));
        else
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s, (k_occ_bucket<OCC_MAX_M / 2, PLACE, false><<<g, b, 0, s>>>(oa)));
    } else {
        if (oa.dtype32)
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s, (k_occ_bucket<OCC_MAX_M, PLACE, true><<<g, b, 0, s>>>(oa)));
        else
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s, (k_occ_bucket<OCC_MAX_M, PLACE, false><<<g, b, 0, s>>>(oa)));
    }
    return SCHULZE_OK;
}

// The accumulation and finish launches for the counter type T of d: packed
// 16-bit LDS counts for unit weights, 32-bit ones otherwise; the LDS row fits
// m; rows read as 32-bit words when the layout allows (WMAX words at most).
template <typename T, int MAXM, bool PACKED>
int occ_accumulate_m(schulze_ctx *ctx, hipStream_t s, const OccArgs &oa, dim3 grid, T *d, int64_t ldd,
                     uint32_t limit, uint8_t *over_flag, int az, int dvec) {
    const dim3 b(256);
    if constexpr (PACKED) {
        if (oa.row_vec == 2 && oa.L <= 32) {
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                           (k_occ_accumulate<MAXM, PACKED, T, 16, true, false><<<grid, b, 0, s>>>(oa, d, ldd, limit, over_flag,
                                                                                          az, dvec)));
            return SCHULZE_OK;
        }
        if (oa.row_vec == 2 && oa.L <= 64) {
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                           (k_occ_accumulate<MAXM, PACKED, T, 32, true, false><<<grid, b, 0, s>>>(oa, d, ldd, limit, over_flag,
                                                                                          az, dvec)));
            return SCHULZE_OK;
        }
        if (oa.row_vec && oa.L <= 32) {
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                           (k_occ_accumulate<MAXM, PACKED, T, 16, false, false><<<grid, b, 0, s>>>(oa, d, ldd, limit, over_flag,
                                                                                           az, dvec)));
            return SCHULZE_OK;
        }
        if (oa.row_vec && oa.L <= 64) {
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                           (k_occ_accumulate<MAXM, PACKED, T, 32, false, false><<<grid, b, 0, s>>>(oa, d, ldd, limit, over_flag,
                                                                                           az, dvec)));
            return SCHULZE_OK;
        }
    }
    if (oa.dtype32)
        SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                       (k_occ_accumulate<MAXM, PACKED, T, 0, false, true><<<grid, b, 0, s>>>(oa, d, ldd, limit,
                                                                                             over_flag, az, dvec)));
    else
        SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                       (k_occ_accumulate<MAXM, PACKED, T, 0, false, false><<<grid, b, 0, s>>>(oa, d, ldd, limit,
                                                                                              over_flag, az, dvec)));
    return SCHULZE_OK;
}

template <typename T>
int occ_accumulate(schulze_ctx *ctx, hipStream_t s, const OccArgs &oa, dim3 grid, int32_t m, bool weighted, T *d,
                   int64_t ldd, uint32_t limit, uint8_t *over_flag, bool acc_zero) {
    const int az = acc_zero ? 1 : 0;
    // rows of d 16-byte aligned: eight columns per 16-byte store (uint16) or two (int32)
    const int dvec = reinterpret_cast<uintptr_t>(d) % 16 == 0 && (ldd * (int64_t)sizeof(T)) % 16 == 0;
    int rc;
    if (!weighted && m <= OCC_MAX_M / 2)
        rc = occ_accumulate_m<T, OCC_MAX_M / 2, true>(ctx, s, oa, grid, d, ldd, limit, over_flag, az, dvec);
    else if (!weighted)
        rc = occ_accumulate_m<T, OCC_MAX_M, true>(ctx, s, oa, grid, d, ldd, limit, over_flag, az, dvec);
    else if (m <= OCC_MAX_M / 2)
        rc = occ_accumulate_m<T, OCC_MAX_M / 2, false>(ctx, s, oa, grid, d, ldd, limit, over_flag, az, dvec);
    else
        rc = occ_accumulate_m<T, OCC_MAX_M, false>(ctx, s, oa, grid, d, ldd, limit, over_flag, az, dvec);
    if (rc != SCHULZE_OK) return rc;
    const dim3 fg((unsigned)(ctx->num_cus * 4));
    if (weighted) {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       (k_occ_finish<T, false><<<fg, dim3(256), 0, s>>>(oa, d, ldd, limit, over_flag, az, dvec)));
    } else {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       (k_occ_finish<T, true><<<fg, dim3(256), 0, s>>>(oa, d, ldd, limit, over_flag, az, dvec)));
    }
    return SCHULZE_OK;
}

constexpr size_t TRUNC_POS_CAP = (size_t)1 << 30;

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
    const int64_t max_pairs = (n + 1) / 2;
    const bool may_have_full = L >= m - 1 && n > 0;
    const bool may_have_trunc = n > 0;  // a row may always end early
    const int64_t upitch_max = round_up((int64_t)m + 1, CT);
    const size_t tpos_bytes = may_have_trunc && !voter_weight
                                  ? std::min(TRUNC_POS_CAP, sizeof(uint32_t) * (size_t)max_pairs * (size_t)upitch_max)
                                  : 0;

    const MetaLayout lay(n, m);
    int rc;
    if ((rc = ws_reserve(ctx, WS_BALLOT_META, lay.total)) != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_ACC32, sizeof(uint32_t) * (size_t)m * m)) != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_ROWSUM, sizeof(uint32_t) * (size_t)m)) != SCHULZE_OK) return rc;
    if (may_have_full &&
        (rc = ws_reserve(ctx, WS_POSITIONS, sizeof(uint32_t) * (size_t)max_pairs * pitch)) != SCHULZE_OK)
        return rc;
    if (tpos_bytes && (rc = ws_reserve(ctx, WS_TRUNC_POS, tpos_bytes)) != SCHULZE_OK) return rc;
    // bucketed pair counting: an LDS row of counts per candidate and a bounded occurrence buffer
    const int64_t occ_cap = n * (int64_t)L;
    const bool occ_ok = n > 0 && m <= OCC_MAX_M && occ_cap <= OCC_MAX && !ctx->legacy_pairs;
    const int64_t occ_grid = (int64_t)ctx->num_cus * (m <= OCC_MAX_M / 2 ? 2 : 1);
    const OccLayout ol(occ_ok ? occ_grid : 0, m, occ_ok ? occ_cap : 0, voter_weight ? 4 : 2);
    if (occ_ok && (rc = ws_reserve(ctx, WS_OCC, ol.total)) != SCHULZE_OK) return rc;

    char *mb = static_cast<char *>(ctx->ws[WS_BALLOT_META]);
    Meta meta{reinterpret_cast<int32_t *>(mb + lay.ctr),
              reinterpret_cast<unsigned long long *>(mb + lay.k2),
              reinterpret_cast<int32_t *>(mb + lay.len),
              reinterpret_cast<int32_t *>(mb + lay.full_src),
              reinterpret_cast<int32_t *>(mb + lay.trunc_src),
              reinterpret_cast<uint8_t *>(mb + lay.in_u),
              reinterpret_cast<int32_t *>(mb + lay.ulist),
              reinterpret_cast<int32_t *>(mb + lay.umap)};
    uint32_t *acc = static_cast<uint32_t *>(ctx->ws[WS_ACC32]);
    uint32_t *rsum = static_cast<uint32_t *>(ctx->ws[WS_ROWSUM]);
    const int64_t lda = m;

    // counters, partial sums and the U bitmap start at zero
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(mb + lay.ctr), (lay.len - lay.ctr) / 4, 0u)) !=
        SCHULZE_OK)
        return rc;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(mb + lay.in_u), (lay.ulist - lay.in_u) / 4, 0u)) !=
        SCHULZE_OK)
        return rc;
    if (n == 0 && (rc = fill_u32(ctx, s, acc, (size_t)m * m, 0u)) != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, rsum, (size_t)m, 0u)) != SCHULZE_OK) return rc;

    uint8_t *over_flag = nullptr;  // the bucketed count's overflow flag (set: it ran and wrote its rows)
    if (n > 0) {
        if (L <= 64) {
            const int64_t per_wg = 4 * SHORT_PER_WAVE * SHORT_ROUNDS * std::min<int64_t>(SHORT_BPW, 64 / L);
            const dim3 sg((unsigned)ceil_div(n, per_wg));
            if (dtype32)
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                               k_scan_short<true><<<sg, dim3(256), 0, s>>>(ballots, n, L, m, meta, ctx->err));
            else
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                               k_scan_short<false><<<sg, dim3(256), 0, s>>>(ballots, n, L, m, meta, ctx->err));
        } else if (!dtype32 && L % 8 == 0 && reinterpret_cast<uintptr_t>(ballots) % 16 == 0) {
            SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                           k_scan_long_vec<<<dim3((unsigned)ceil_div(n, LONG_CHUNK)), dim3(256), 0, s>>>(
                               static_cast<const uint16_t *>(ballots), n, L, m, meta, ctx->err));
        } else {
            const dim3 lg((unsigned)ceil_div(n, LONG_CHUNK));
            if (dtype32)
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                               k_scan_long<true><<<lg, dim3(256), 0, s>>>(ballots, n, L, m, meta, ctx->err));
            else
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCAN, s,
                               k_scan_long<false><<<lg, dim3(256), 0, s>>>(ballots, n, L, m, meta, ctx->err));
        }
        SCHULZE_LAUNCH(ctx, K_ROUTE, s,
                       k_route<<<dim3(1), dim3(ROUTE_THREADS), 0, s>>>(m, meta, voter_weight != nullptr,
                                                             (int64_t)(tpos_bytes / sizeof(uint32_t)),
                                                             occ_ok ? BUCKETED_PAIR_COST : ATOMIC_PAIR_COST));
        {
            // the m x m accumulator starts at zero unless the device chose the
            // bucketed route and there are no full rankings: then nothing reads it
            const int64_t words = (int64_t)m * m;
            const unsigned fg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(words / 4 + 1, 256),
                                                                                 (int64_t)ctx->num_cus * 8));
            SCHULZE_LAUNCH(ctx, K_FILL, s,
                           k_fill_acc<<<dim3(fg), dim3(256), 0, s>>>(acc, words, meta, occ_ok && !may_have_full ? 1 : 0));
        }
        if (voter_weight) {
            // counters 32..33: the 64-bit total; 34: workgroups done (zeroed above)
            const unsigned tg = (unsigned)std::min<int64_t>(ceil_div(n, 256), (int64_t)ctx->num_cus * 4);
            SCHULZE_LAUNCH(ctx, K_ROUTE, s,
                           k_weight_total<<<dim3(tg), dim3(256), 0, s>>>(
                               voter_weight, n, reinterpret_cast<unsigned long long *>(meta.ctr + 32), meta.ctr + 34,
                               ctx->err));
        }
        const unsigned cgrid = (unsigned)ctx->num_cus * 2;
        const unsigned scatter_grid = (unsigned)std::min<int64_t>(max_pairs, (int64_t)ctx->num_cus * 16);
        if (may_have_full) {
            uint32_t *pos = static_cast<uint32_t *>(ctx->ws[WS_POSITIONS]);
            if (dtype32)
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCATTER, s,
                               k_scatter<true, true><<<dim3(scatter_grid), dim3(256), 0, s>>>(
                                   ballots, L, m, pitch, meta, pos, ctx->err));
            else
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCATTER, s,
                               k_scatter<true, false><<<dim3(scatter_grid), dim3(256), 0, s>>>(
                                   ballots, L, m, pitch, meta, pos, ctx->err));
            if (!voter_weight) {
                DenseArgs da{pos, pitch, m, meta, acc, lda, rsum};
                SCHULZE_LAUNCH(ctx, K_COUNT_DENSE, s, k_count_pos<false><<<dim3(cgrid), dim3(CNT_THREADS), 0, s>>>(da));
            } else {
                dim3 grid((unsigned)ceil_div(m, 16), (unsigned)ceil_div(m, 16));
                SCHULZE_LAUNCH(ctx, K_COUNT_DENSE, s,
                               k_count_full_weighted<<<grid, dim3(256), 0, s>>>(voter_weight, meta, pos, pitch, m, acc,
                                                                               lda));
            }
        }
        if (tpos_bytes) {
            uint32_t *tpos = static_cast<uint32_t *>(ctx->ws[WS_TRUNC_POS]);
            if (dtype32)
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCATTER, s,
                               k_scatter<false, true><<<dim3(scatter_grid), dim3(256), 0, s>>>(
                                   ballots, L, m, 0, meta, tpos, ctx->err));
            else
                SCHULZE_LAUNCH(ctx, K_BALLOT_SCATTER, s,
                               k_scatter<false, false><<<dim3(scatter_grid), dim3(256), 0, s>>>(
                                   ballots, L, m, 0, meta, tpos, ctx->err));
            DenseArgs da{tpos, 0, m, meta, acc, lda, rsum};
            SCHULZE_LAUNCH(ctx, K_COUNT_TRUNC, s, k_count_pos<true><<<dim3(cgrid), dim3(CNT_THREADS), 0, s>>>(da));
        }
        if (occ_ok) {
            // bucketed pair counting (runs only if the device chose pair scattering)
            char *ob = static_cast<char *>(ctx->ws[WS_OCC]);
            int32_t tbits = 0;
            while ((1 << tbits) < L) ++tbits;
            const bool pieces = reinterpret_cast<uintptr_t>(ballots) % 16 == 0 && (n * L) % 8 == 0;
            const int row_vec =
                !dtype32 && L % 2 == 0 && reinterpret_cast<uintptr_t>(ballots) % 4 == 0 ? (pieces ? 2 : 1) : 0;
            OccArgs oa{ballots, dtype32, L, m, n, tbits, row_vec, voter_weight, meta,
                       reinterpret_cast<uint32_t *>(ob + ol.hist),
                       reinterpret_cast<uint32_t *>(ob + ol.row_start),
                       reinterpret_cast<uint32_t *>(ob + ol.item_start),
                       reinterpret_cast<uint32_t *>(ob + ol.part_start),
                       reinterpret_cast<int32_t *>(ob + ol.fin),
                       reinterpret_cast<uint32_t *>(ob + ol.occ),
                       static_cast<void *>(ob + ol.partial), ol.ppitch,
                       acc, lda, rsum, ctx->err};
            const dim3 g(occ_grid);
            over_flag = reinterpret_cast<uint8_t *>(ob + ol.over_flag);
            if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(over_flag), 1, 0u)) !=
                SCHULZE_OK)
                return rc;
            if ((rc = occ_bucket<false>(ctx, s, oa, g)) != SCHULZE_OK) return rc;
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                           k_occ_columns<<<dim3((unsigned)ceil_div(m, 64)), dim3(64 * COL_GROUPS), 0, s>>>(
                               oa, (int32_t)occ_grid));
            SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s, k_occ_scan<<<dim3(1), dim3(1024), 0, s>>>(oa));
            const dim3 ig((unsigned)(m + ceil_div(occ_cap, OCC_CHUNK)));
            if ((rc = occ_bucket<true>(ctx, s, oa, g)) != SCHULZE_OK) return rc;
            if (d_dtype == SCHULZE_U16) {
                if ((rc = occ_accumulate<uint16_t>(ctx, s, oa, ig, m, voter_weight != nullptr, (uint16_t *)d, ldd,
                                                   65535u, over_flag, !may_have_full)) != SCHULZE_OK)
                    return rc;
            } else {
                if ((rc = occ_accumulate<int32_t>(ctx, s, oa, ig, m, voter_weight != nullptr, (int32_t *)d, ldd,
                                                  (uint32_t)INT32_MAX, over_flag, !may_have_full)) != SCHULZE_OK)
                    return rc;
            }
        } else {
            const dim3 pg((unsigned)ceil_div(n, 4));
            if (dtype32)
                SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                               k_count_pairs<true><<<pg, dim3(256), 0, s>>>(ballots, L, m, voter_weight, meta, acc, lda,
                                                                            rsum, ctx->err));
            else
                SCHULZE_LAUNCH(ctx, K_COUNT_SPARSE, s,
                               k_count_pairs<false><<<pg, dim3(256), 0, s>>>(ballots, L, m, voter_weight, meta, acc,
                                                                             lda, rsum, ctx->err));
        }
    }
    // rows of the bucketed route were written by it (over_flag given)
    dim3 fgrid((unsigned)m);
    if (d_dtype == SCHULZE_U16) {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       k_count_finish<uint16_t><<<fgrid, dim3(256), 0, s>>>(acc, lda, rsum, meta, m, (uint16_t *)d, ldd,
                                                                            65535u, ctx->err, over_flag != nullptr));
    } else {
        SCHULZE_LAUNCH(ctx, K_COUNT_FINISH, s,
                       k_count_finish<int32_t><<<fgrid, dim3(256), 0, s>>>(acc, lda, rsum, meta, m, (int32_t *)d, ldd,
                                                                           (uint32_t)INT32_MAX, ctx->err,
                                                                           over_flag != nullptr));
    }
    return SCHULZE_OK;
}
