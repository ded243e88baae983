// Batched elections in one persistent launch.
//
// Every election of a batch is one Schulze instance (Section 2.1): its own
// profile, counts d, widest-path closure p, winners and ranking.  A host
// plan turns the batch into a queue of work items; the workgroups of one
// persistent kernel take items in queue order from an atomic ticket:
//
//   scan    ballots of one range of voters -> rank pairs (the ranks of two
//           voters in one 32-bit word, low half the even voter), checked for
//           ids out of range, repeated ids and ids after padding;
//   count   one run of up to 256 sub-blocks of 8 x 8 candidates of one
//           election over one range of voters.  For a pair (x, y) and a
//           voter, t = (rank(x) - rank(y)) mod 2^16 equals
//           rank(x) - rank(y) + 2^16 [rank(x) < rank(y)], so summed over
//           voters  sum t = Sx - Sy + 2^16 #(x before y)  with Sx the sum of
//           x's ranks: one v_pk_sub_u16 and one v_dot2_u32_u16 handle two
//           voters.  Complete rankings have no ties, so only sub-blocks with
//           x-block <= y-block are counted and d[y][x] = voters - d[x][y];
//           elections with truncated ballots count every ordered sub-block;
//   finish  edge weights, closure, beaten-by counts, winners and ranking of
//           one election in one workgroup, started by the workgroup that
//           completes the election's last count item.
//
// The scans of an election come before its counts in the queue (a few
// elections ahead, so that memory-bound scans overlap VALU-bound counts).  A
// count item waits only for the scans of its own election, whose tickets are
// smaller and are held by workgroups that are already running and never
// wait, so every wait ends however many workgroups are resident.  A bounded
// spin turns anything else into a device error.
//
// The closure of the finish runs on a per-workgroup scratch matrix of uint16
// (counts of elections with at most 65535 voters) or int32, padded with zero
// rows and columns, by one of two schedules chosen per election size:
// REGISTERS, the plain recurrence with the whole padded matrix (up to
// 192 x 192 uint16 or 128 x 128 int32) held in registers, or TILED(B), the
// three-phase blocked recurrence with B x B tiles run by one workgroup
// (B = 32 and 128 for uint16 only).
#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "fw_tiles.h"

namespace {

using namespace fw;

constexpr int BT = 256;                          // threads per workgroup
constexpr int STAGE_WORDS = 16384;               // count staging: VC x cols words
constexpr int SRED_WORDS = SCHULZE_BATCH_MAX_M;  // column sums of a count item
constexpr int SMEM_WORDS = STAGE_WORDS + SRED_WORDS + 64;
constexpr int SEG_PAIRS = 32767;           // at most 65534 voters per exact sum
constexpr int64_t SCAN_WORDS = 1 << 20;    // rank-pair words written per scan item
constexpr int SCAN_GROUP_WORDS = 16384;    // rank-pair words staged at once by a scan
constexpr int SCAN_VEC = 16;              // 16-byte ballot loads in flight per thread
constexpr int SCAN_GROUP_PAIRS = 32;      // voter pairs staged at once by a scan, at most
constexpr int MAX_PF = 8;                  // 16-byte loads per thread per count chunk
constexpr uint16_t UNSET = 0xFFFF;
constexpr int64_t SPIN_LIMIT = (int64_t)1 << 24;

enum ItemKind : int32_t { IT_SCAN = 0, IT_COUNT = 1, IT_FINISH = 2 };
enum ElecFlags : int32_t { EF_SQUARE = 1, EF_MULTI = 2, EF_VAL16 = 4, EF_ZERO_D = 8 };

// Per-election parameters (host plan -> device).
struct BElec {
    int64_t ballot_off;  // elements
    int64_t n;           // voters
    int64_t mat_off;     // elements of d and p
    int64_t vec_off;     // elements of is_winner, beaten_by, order
    int64_t pos_off;     // rank-pair words
    int32_t m, L;
    int32_t pitch;        // rank-pair words per voter pair (= 8 * nb8)
    int32_t flags;        // ElecFlags
    int32_t n_scan;       // scan items
    int32_t n_count;      // count items
    int32_t variant;      // closure schedule
    int32_t mp;           // padded closure size
    int32_t nb8;          // blocks of 8 candidates
    int32_t vc;           // voter pairs per staged chunk (64 / ng)
    int32_t ng;           // column groups of 64 quads in a staged row (1, 2 or 4)
    int32_t vs;           // voter split of small elections (1, 2 or 4)
    int32_t range_pairs;  // voter pairs per count range
    int32_t scan_pairs;   // voter pairs per scan item
};
static_assert(sizeof(BElec) == 96, "BElec layout");

struct BItem {
    int32_t kind, e, a, b;  // scan: a = first voter pair, b = pairs; count: a = run, b = range
};

struct BatchArgs {
    const BElec *elec;
    const BItem *items;
    int32_t n_items;
    int32_t n_elec;
    const void *ballots;
    int32_t dtype32;
    int32_t mode;
    int32_t closure_only;
    int32_t pad0;
    uint32_t *pos;
    int32_t *d;
    int32_t *p;
    uint8_t *is_winner;
    int32_t *n_winners;
    int32_t *beaten_by;
    int32_t *order;
    int32_t *level;  // NULL or top-k levels (-1 = not reached)
    int32_t topk;    // rank at least this many candidates per election (0: no levels)
    int32_t pad1;
    int32_t *ctr;  // [0] ticket, [1] abort, [2, 2+E) scans done, [2+E, 2+2E) counts done
    char *scratch;
    int64_t scratch_bytes;  // per workgroup
    int32_t *err;
};

// Every device-memory access of this file goes through FW_GLOBAL pointers, so
// that it compiles to global_* instructions: flat ones would also count as
// LDS operations and every LDS wait would then wait for them too.
template <typename T>
__device__ __forceinline__ FW_GLOBAL T *gmem(T *p) {
    return (FW_GLOBAL T *)p;
}

// LDS of the persistent kernel, used by every function below.  Static (not
// dynamic) so that its address is a constant in every function; a dynamic
// array is located through a table lookup in functions that are not kernels.
__shared__ __attribute__((aligned(16))) uint32_t batch_smem[SMEM_WORDS];

// Candidate id of a ballot entry, -1 for padding.
__device__ inline int32_t ballot_id(int32_t v) { return v < 0 ? -1 : v; }
__device__ inline int32_t ballot_id(uint16_t v) { return v == 0xFFFF ? -1 : (int32_t)v; }

// floor(x / d) for 0 <= x < 2^16 and 1 <= d <= 2^16, with inv = ceil(2^32 / d):
// the error x * (inv - 2^32/d) / 2^32 < 2^-16 <= 1/d never crosses an integer.
__device__ inline uint32_t div_small(uint32_t x, uint32_t inv) { return __umulhi(x, inv); }

__host__ __device__ inline int32_t scan_group_pairs(int32_t pitch) {
    return SCAN_GROUP_WORDS / pitch < SCAN_GROUP_PAIRS ? SCAN_GROUP_WORDS / pitch : SCAN_GROUP_PAIRS;
}

__device__ inline void abort_all(const BatchArgs &a) {
    __hip_atomic_store(gmem(a.ctr) + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    set_device_error(a.err, SCHULZE_EDEVICE);
}

// ------------------------------------------------------------------ scan
// Voter pairs [q0, q0 + nq) of one election, SCAN_GROUP_WORDS words at a time.
// A ballot lists k = (index of its first padding entry) candidates; it is
// valid iff no id follows a padding entry, every listed id is < m, and the
// listed ids leave exactly m - k candidates unset (no repeats).  Complete
// elections (L >= m - 1) also need k >= m - 1: their unset candidate is last.
template <typename Id>
__device__ __attribute__((noinline)) void scan_item(const BatchArgs &a, const BElec &el_in, int64_t q0, int64_t nq) {
    // Local copies: a re-read through the references would be a flat load,
    // and every flat load waits for all outstanding global loads.
    const BElec el = el_in;
    uint32_t *smem = batch_smem;
    const FW_GLOBAL Id *ballots = gmem(static_cast<const Id *>(a.ballots));
    const int tid = threadIdx.x;
    const int32_t m = el.m, L = el.L, pitch = el.pitch;
    const bool complete = (el.flags & EF_SQUARE) == 0;
    const int32_t vpb = scan_group_pairs(pitch);  // voter pairs per group, 8 .. SCAN_GROUP_PAIRS
    uint16_t *buf = reinterpret_cast<uint16_t *>(smem);
    int32_t *first_pad = reinterpret_cast<int32_t *>(smem + SCAN_GROUP_WORDS);  // [2 vpb]
    int32_t *npads = first_pad + 64;
    int32_t *unset = npads + 64;
    const uint32_t inv_l = L > 1 ? (uint32_t)((0x100000000ull + (uint64_t)L - 1) / (uint64_t)L) : 0u;
    const uint32_t inv_p = (uint32_t)((0x100000000ull + (uint64_t)pitch - 1) / (uint64_t)pitch);
    FW_GLOBAL uint32_t *pos = gmem(a.pos + el.pos_off);

    if ((el.flags & EF_MULTI) && q0 == 0) {  // counts accumulate with atomics: start at zero
        FW_GLOBAL int32_t *D = gmem(a.d + el.mat_off);
        for (int64_t i = tid; i < (int64_t)m * m; i += BT) D[i] = 0;
    }
    bool bad = false;
    for (int64_t g = q0; g < q0 + nq; g += vpb) {
        const int32_t npg = (int32_t)min((int64_t)vpb, q0 + nq - g);
        const int64_t v0 = 2 * g;  // first voter of the group
        const int32_t nballots = (int32_t)min((int64_t)2 * npg, el.n - v0);
        const int32_t nquads = npg * pitch / 4;  // pitch is a multiple of 8
        __syncthreads();
        for (int32_t w4 = tid; w4 < nquads; w4 += BT)
            reinterpret_cast<v4u32 *>(smem)[w4] = v4u32{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        if (tid < 2 * vpb) {
            first_pad[tid] = L;
            npads[tid] = 0;
            unset[tid] = 0;
        }
        __syncthreads();
        const int64_t base = el.ballot_off + v0 * (int64_t)L;  // ballots of the group are contiguous
        const int32_t entries = nballots * L;                // < 2^16
        // entry f of the group: id -> LDS (ballot b = f / L at position t)
        auto take = [&](int32_t f, int32_t id) {
            const int32_t b = (int32_t)div_small((uint32_t)f, inv_l) + (L == 1 ? f : 0);  // inv_l = 0 if L = 1
            const int32_t t = f - b * L;
            bad |= id >= m;
            if ((uint32_t)id < (uint32_t)m) buf[(b >> 1) * 2 * pitch + 2 * id + (b & 1)] = (uint16_t)t;
            if (id < 0) {  // padding: rare, and never in complete elections' valid ballots
                atomicAdd(&npads[b], 1);
                atomicMin(&first_pad[b], t);
            }
        };
        // 16-byte loads over the aligned span that covers the entries (its
        // head lies inside the ballot array before them and is skipped), the
        // last partial vector entry by entry; SCAN_VEC loads in flight per
        // thread, issued unconditionally (clamped) before any is used
        constexpr int V = 16 / (int)sizeof(Id);
        const int64_t a0 = base & ~(int64_t)(V - 1);
        const int64_t end = base + entries;
        const int64_t vend = end & ~(int64_t)(V - 1);
        const int32_t nvec = vend > a0 ? (int32_t)((vend - a0) / V) : 0;
        const FW_GLOBAL v4u32 *bv = (const FW_GLOBAL v4u32 *)(ballots + a0);
        for (int32_t k0 = tid; k0 < nvec; k0 += BT * SCAN_VEC) {
            v4u32 raw[SCAN_VEC];
#pragma unroll
            for (int j = 0; j < SCAN_VEC; ++j) {
                const int32_t k = k0 + BT * j;
                raw[j] = bv[k < nvec ? k : nvec - 1];
            }
#pragma unroll
            for (int j = 0; j < SCAN_VEC; ++j) {
                const int32_t k = k0 + BT * j;
                if (k >= nvec) break;
                const uint32_t w[4] = {raw[j].x, raw[j].y, raw[j].z, raw[j].w};
                const int32_t f0 = (int32_t)(a0 + (int64_t)k * V - base);  // entry of the first id (may be < 0)
                auto id_of = [&](int u) -> int32_t {
                    if constexpr (sizeof(Id) == 2)
                        return ballot_id((uint16_t)((w[u >> 1] >> ((u & 1) * 16)) & 0xFFFFu));
                    else
                        return ballot_id((int32_t)w[u]);
                };
                if (f0 >= 0 && f0 + V <= entries) {
                    // whole vector inside the group: ballot and position once, then stepped
                    int32_t b = (int32_t)div_small((uint32_t)f0, inv_l) + (L == 1 ? f0 : 0);
                    int32_t t = f0 - b * L;
                    int32_t row = (b >> 1) * 2 * pitch + (b & 1);
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int32_t id = id_of(u);
                        if ((uint32_t)id < (uint32_t)m)
                            buf[row + 2 * id] = (uint16_t)t;
                        else
                            take(f0 + u, id);  // padding or out of range
                        if (++t == L) {
                            t = 0;
                            ++b;
                            row = (b >> 1) * 2 * pitch + (b & 1);
                        }
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int32_t f = f0 + u;
                        if (f >= 0 && f < entries) take(f, id_of(u));
                    }
                }
            }
        }
        // entries after the last whole vector
        {
            const int64_t t0 = vend > base ? vend : base;
            const int32_t nt = (int32_t)(end - t0);
            if (tid < nt) take((int32_t)(t0 + tid - base), ballot_id(ballots[t0 + tid]));
        }
        __syncthreads();
        // four words per thread: one voter pair's columns c .. c+3 (pitch is a multiple of 8)
        for (int32_t w4 = tid; w4 < nquads; w4 += BT) {
            const int32_t w = 4 * w4;
            const int32_t q = (int32_t)div_small((uint32_t)w, inv_p);
            const int32_t c0 = w - q * pitch;
            const bool has_hi = 2 * q + 1 < nballots;
            const v4u32 in4 = reinterpret_cast<const v4u32 *>(smem)[w4];
            const uint32_t words[4] = {in4.x, in4.y, in4.z, in4.w};
            uint32_t out[4];
            int32_t un_lo = 0, un_hi = 0;
            if (c0 + 4 <= m) {  // all four columns are candidates
                const uint32_t fill = complete ? (uint32_t)(m - 1) : UNSET;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t lo = words[e] & 0xFFFFu, hi = words[e] >> 16;
                    const bool ul = lo == UNSET, uh = hi == UNSET;
                    un_lo += ul ? 1 : 0;
                    un_hi += uh ? 1 : 0;
                    lo = ul ? fill : lo;
                    hi = uh ? fill : hi;
                    out[e] = lo | (hi << 16);
                }
                if (!has_hi) {  // missing partner of an odd count: equal ranks, counts nothing
                    un_hi = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) out[e] &= 0xFFFFu;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t lo = words[e] & 0xFFFFu, hi = words[e] >> 16;
                    if (c0 + e < m) {
                        un_lo += lo == UNSET ? 1 : 0;
                        un_hi += (has_hi && hi == UNSET) ? 1 : 0;
                        if (complete) {
                            if (lo == UNSET) lo = (uint32_t)(m - 1);
                            if (hi == UNSET) hi = (uint32_t)(m - 1);
                        }
                    } else {
                        lo = hi = 0u;
                    }
                    if (!has_hi) hi = 0u;
                    out[e] = lo | (hi << 16);
                }
            }
            if (un_lo) atomicAdd(&unset[2 * q], un_lo);
            if (un_hi) atomicAdd(&unset[2 * q + 1], un_hi);
            *(FW_GLOBAL v4u32 *)(pos + (g + q) * (int64_t)pitch + c0) = v4u32{out[0], out[1], out[2], out[3]};
        }
        __syncthreads();
        if (tid < nballots) {
            const int32_t k = first_pad[tid];
            if (L - npads[tid] != k || unset[tid] != m - k || (complete && k < m - 1)) bad = true;
        }
    }
    if (bad) set_device_error(a.err, SCHULZE_EBALLOT);
}

// ------------------------------------------------------------------ count
__device__ inline void sub_coords(int32_t s, int32_t nb8, bool square, int32_t &bx, int32_t &by) {
    if (square) {
        bx = s / nb8;
        by = s - bx * nb8;
        return;
    }
    int32_t x = 0, start = 0;
    while (start + (nb8 - x) <= s) {
        start += nb8 - x;
        ++x;
    }
    bx = x;
    by = x + (s - start);
}

typedef __attribute__((ext_vector_type(2))) unsigned short cus2;

__device__ void finish(const BatchArgs &a, const BElec &el, int32_t e);

// Sub-blocks [run * per_phase, ...) of election e over voter pairs of range
// `range`.  Staged rows hold columns c0 .. 8 nb8 - 1 of VC voter pairs, each
// 8-column block split into two 16-byte halves stored in separate row
// halves so that neighbouring sub-blocks read neighbouring 16 bytes.
__device__ __attribute__((noinline)) void count_item(const BatchArgs &a, const BElec &el_in, int32_t e, int32_t run,
                                                    int32_t range) {
    const BElec el = el_in;  // local copy (see scan_item)
    const int64_t pitch = el.pitch;
    uint32_t *smem = batch_smem;
    __shared__ int32_t sh_flag;
    const int tid = threadIdx.x;
    const bool square = (el.flags & EF_SQUARE) != 0;
    const bool multi = (el.flags & EF_MULTI) != 0;
    const int32_t m = el.m, nb8 = el.nb8;
    const int32_t vs = el.vs, per_phase = BT / vs;
    const int32_t phase = tid / per_phase, lt = tid - phase * per_phase;
    const int32_t S = square ? nb8 * nb8 : nb8 * (nb8 + 1) / 2;
    const int32_t s_first = run * per_phase;
    const int32_t s_mine = s_first + lt;
    const bool active = s_mine < S;
    int32_t bx0, by0;
    sub_coords(s_first, nb8, square, bx0, by0);
    const int32_t cb0 = square ? 0 : bx0;  // first staged block of 8 columns
    int32_t bx = cb0, by = cb0;
    if (active) sub_coords(s_mine, nb8, square, bx, by);
    const int32_t c0 = 8 * cb0;
    const int32_t cols = 8 * (nb8 - cb0);
    const int32_t half = cols / 2;
    const int32_t nq = cols / 4;  // 16-byte quads per staged row
    const int32_t ng = el.ng, lg = ng == 1 ? 0 : (ng == 2 ? 1 : 2);
    const int32_t VC = el.vc;  // 4 MAX_PF / ng: VC * cols <= STAGE_WORDS, ng * VC / 4 == MAX_PF
    const int64_t pairs = (el.n + 1) / 2;
    const int64_t p0 = (int64_t)range * el.range_pairs;
    const int64_t p1 = min(pairs, p0 + el.range_pairs);
    const uint32_t nv = (uint32_t)(min(el.n, 2 * p1) - 2 * p0);
    const FW_GLOBAL uint32_t *pos = gmem(a.pos + el.pos_off);
    uint32_t *stage = smem;
    uint32_t *sred = smem + STAGE_WORDS;
    const int32_t qlane = tid & 63, prow = tid >> 6;

    // the scans of this election must be complete
    if (tid == 0) {
        int32_t ok = 1;
        int64_t spins = 0;
        FW_GLOBAL int32_t *ctr = gmem(a.ctr);
        while (__hip_atomic_load(ctr + 2 + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < el.n_scan) {
            if (__hip_atomic_load(ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > SPIN_LIMIT) {
                abort_all(a);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        sh_flag = ok;
    }
    __syncthreads();
    if (!sh_flag) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    uint32_t acc[8][8];
    uint32_t scol[4][4];
    v4u32 pf[MAX_PF];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) scol[i][j] = 0u;

    // slot k holds quad qlane + 64 (k & (ng-1)) of voter pair prow + 4 (k >> lg)
    // Unconditional loads, so that all MAX_PF are in flight at once: a slot
    // outside the chunk reads the election's first word, and stage_store
    // writes zeros for it instead.
    auto slot_ok = [&](int k, int64_t q0) {
        return qlane + 64 * (k & (ng - 1)) < nq && q0 + prow + 4 * (k >> lg) < p1;
    };
    auto prefetch = [&](int64_t q0) {
#pragma unroll
        for (int k = 0; k < MAX_PF; ++k) {
            const int32_t qd = qlane + 64 * (k & (ng - 1));
            const int64_t pr = q0 + prow + 4 * (k >> lg);
            pf[k] = *(const FW_GLOBAL v4u32 *)(pos + (slot_ok(k, q0) ? pr * pitch + c0 + 4 * qd : 0));
        }
    };
    const cus2 ones = {1, 1};
    auto stage_store = [&](int64_t q0, uint32_t *stb) {
#pragma unroll
        for (int k = 0; k < MAX_PF; ++k) {
            const int32_t qd = qlane + 64 * (k & (ng - 1));
            const int32_t vp = prow + 4 * (k >> lg);
            if (qd < nq) {
                const v4u32 v = slot_ok(k, q0) ? pf[k] : v4u32{0u, 0u, 0u, 0u};
                *reinterpret_cast<v4u32 *>(stb + vp * cols + (qd & 1) * half + (qd >> 1) * 4) = v;
                // words through scalars: a bit_cast of an element of a vector value
                // has compiled to the first element here
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    scol[k & 3][q] = __builtin_amdgcn_udot2(__builtin_bit_cast(cus2, w[q]), ones, scol[k & 3][q], false);
            }
        }
    };

    // Two stage buffers (VC * cols <= 8192 words each): chunk c is counted
    // from one while chunk c+1 is written to the other, one barrier per chunk.
    const int32_t xo = (bx - cb0) * 4, yo = (by - cb0) * 4;
    uint32_t *const stage_b[2] = {stage, stage + VC * cols};
    prefetch(p0);
    __syncthreads();  // the stage is free (a previous item of this workgroup may have used it)
    stage_store(p0, stage_b[0]);
    __syncthreads();
    int cur = 0;
    for (int64_t q0 = p0; q0 < p1; q0 += VC) {
        const bool more = q0 + VC < p1;
        if (more) prefetch(q0 + VC);  // overlaps the compute below
        const uint32_t *st = cur ? stage_b[1] : stage_b[0];  // (select: a dynamically indexed array would live in scratch)
        const int32_t vend = (int32_t)min((int64_t)VC, p1 - q0);
        if (active) {
#pragma unroll 1
            for (int32_t v = phase; v < vend; v += vs) {
                const uint32_t *row = st + v * cols;
                const uint4 xa = *reinterpret_cast<const uint4 *>(row + xo);
                const uint4 xb = *reinterpret_cast<const uint4 *>(row + half + xo);
                const uint4 ya = *reinterpret_cast<const uint4 *>(row + yo);
                const uint4 yb = *reinterpret_cast<const uint4 *>(row + half + yo);
                const uint32_t xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
                const uint32_t yv[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const cus2 xi = __builtin_bit_cast(cus2, xv[i]);
                    cus2 diff[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) diff[j] = xi - __builtin_bit_cast(cus2, yv[j]);
#pragma unroll
                    for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_udot2(diff[j], ones, acc[i][j], false);
                }
            }
        }
        if (more) stage_store(q0 + VC, cur ? stage_b[0] : stage_b[1]);
        __syncthreads();  // the next chunk is staged; everyone is done with this one
        cur ^= 1;
    }

    // column sums of the range, then the counts
    __syncthreads();
    for (int32_t c = tid; c < cols; c += BT) sred[c] = 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int32_t qd = qlane + 64 * (j & (ng - 1));
        if (qd < nq) {
            // slots j, j+4, ... of this thread all hold quad qd
            const int32_t col = 4 * qd;  // first staged column of the quad
#pragma unroll
            for (int q = 0; q < 4; ++q) atomicAdd(&sred[col + q], scol[j][q]);
        }
    }
    if (vs > 1 && phase > 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) stage[((phase - 1) * 64 + i * 8 + j) * per_phase + lt] = acc[i][j];
    }
    __syncthreads();
    if (phase == 0 && active) {
        if (vs > 1) {
            for (int32_t ph = 1; ph < vs; ++ph)
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) acc[i][j] += stage[((ph - 1) * 64 + i * 8 + j) * per_phase + lt];
        }
        uint32_t sx[8], sy[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) sx[i] = sred[8 * (bx - cb0) + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) sy[j] = sred[8 * (by - cb0) + j];
        FW_GLOBAL int32_t *D = gmem(a.d + el.mat_off);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int32_t x = 8 * bx + i;
            if (x >= m) continue;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t y = 8 * by + j;
                if (y >= m) continue;
                const uint32_t cnt = (acc[i][j] - sx[i] + sy[j]) >> 16;
                if (square) {
                    if (x == y) {
                        if (!multi) D[(int64_t)x * m + y] = 0;
                    } else if (multi) {
                        __hip_atomic_fetch_add(D + (int64_t)x * m + y, (int32_t)cnt, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        D[(int64_t)x * m + y] = (int32_t)cnt;
                    }
                } else if (x < y) {
                    if (multi) {
                        __hip_atomic_fetch_add(D + (int64_t)x * m + y, (int32_t)cnt, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_add(D + (int64_t)y * m + x, (int32_t)(nv - cnt), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        D[(int64_t)x * m + y] = (int32_t)cnt;
                        D[(int64_t)y * m + x] = (int32_t)(nv - cnt);
                    }
                } else if (x == y && !multi) {
                    D[(int64_t)x * m + x] = 0;
                }
            }
        }
    }

    // completion: the workgroup that finishes the election's last count item runs its finish
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0)
        sh_flag = __hip_atomic_fetch_add(gmem(a.ctr) + 2 + a.n_elec + e, 1, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) == el.n_count - 1;
    __syncthreads();
    if (sh_flag) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        finish(a, el, e);
    }
}

// ------------------------------------------------------------------ finish
// Blocked recurrence of one workgroup over an mp x mp matrix (mp a multiple
// of B): per round r the diagonal tile is closed, then the panels of block
// row and column r, then the rest; every tile becomes
// max(P[I][J], P[I][r] (x) P[r][J]).
template <typename E, int B>
__device__ __attribute__((noinline)) void closure_tiled(E *P_, int32_t mp) {
    FW_GLOBAL E *P = gmem(P_);
    E *lds = reinterpret_cast<E *>(batch_smem);
    const int32_t nb = mp / B;
    auto tile = [&](int32_t I, int32_t J) { return P + (int64_t)I * B * mp + (int64_t)J * B; };
    for (int32_t r = 0; r < nb; ++r) {
        diag_close<E, B>(tile(r, r), mp, tile(r, r), mp, nullptr, 0, lds);
        for (int32_t t = 0; t < 2 * (nb - 1); ++t) {
            int32_t I, J;
            if (t < nb - 1) {
                I = r;
                J = t < r ? t : t + 1;
            } else {
                const int32_t u = t - (nb - 1);
                J = r;
                I = u < r ? u : u + 1;
            }
            Acc<E, B> acc;
            acc_load<E, B>(acc, tile(I, J), mp);
            acc_product<E, B>(acc, tile(I, r), mp, tile(r, J), mp, lds);
            acc_store<E, B>(acc, tile(I, J), mp);
        }
        for (int32_t t = 0; t < (nb - 1) * (nb - 1); ++t) {
            const int32_t i = t / (nb - 1), j = t % (nb - 1);
            const int32_t I = i < r ? i : i + 1, J = j < r ? j : j + 1;
            Acc<E, B> acc;
            acc_load<E, B>(acc, tile(I, J), mp);
            acc_product<E, B>(acc, tile(I, r), mp, tile(r, J), mp, lds);
            acc_store<E, B>(acc, tile(I, J), mp);
        }
        __syncthreads();
    }
}

static_assert(2 * 4 * MAX_PF * 64 * 4 <= STAGE_WORDS, "two count stage buffers: VC * cols <= 32 / ng * 256 ng words each");
static_assert(diag_lds_elems<uint16_t, 192>() * 2 <= SMEM_WORDS * 4 && diag_lds_elems<int32_t, 128>() * 4 <= SMEM_WORDS * 4,
              "diagonal closure LDS");

// Each schedule is its own function: inlined together, their register
// demands would be allocated as one and spill.
template <typename E, int B>
__device__ __attribute__((noinline)) void closure_reg(E *P_, int32_t mp) {
    FW_GLOBAL E *P = gmem(P_);
    diag_close<E, B>(P, mp, P, mp, nullptr, 0, reinterpret_cast<E *>(batch_smem));
}

template <typename E>
__device__ void closure_dispatch(E *P, int32_t mp, int32_t variant) {
    if (variant == SCHULZE_BATCH_CLOSURE_REGISTERS) {
        switch (mp) {
            case 32: closure_reg<E, 32>(P, mp); break;
            case 64: closure_reg<E, 64>(P, mp); break;
            case 96: closure_reg<E, 96>(P, mp); break;
            case 128: closure_reg<E, 128>(P, mp); break;
            default:
                if constexpr (sizeof(E) == 2) {
                    switch (mp) {
                        case 160: closure_reg<E, 160>(P, mp); break;
                        case 192: closure_reg<E, 192>(P, mp); break;
                        default: break;
                    }
                }
                break;
        }
    } else if (variant == SCHULZE_BATCH_CLOSURE_TILED32) {
        if constexpr (sizeof(E) == 2) closure_tiled<E, 32>(P, mp);
    } else if (variant == SCHULZE_BATCH_CLOSURE_TILED64) {
        closure_tiled<E, 64>(P, mp);
    } else {
        if constexpr (sizeof(E) == 2) closure_tiled<E, 128>(P, mp);
    }
}

template <typename E>
__device__ void finish_t(const BatchArgs &a, const BElec &el, int32_t e, uint32_t *smem) {
    const int tid = threadIdx.x;
    const int32_t m = el.m, mp = el.mp;
    const int32_t mode = a.mode;
    FW_GLOBAL uint8_t *is_winner = gmem(a.is_winner);
    FW_GLOBAL int32_t *beaten_by = a.beaten_by ? gmem(a.beaten_by) : nullptr;
    FW_GLOBAL int32_t *order = a.order ? gmem(a.order) : nullptr;
    FW_GLOBAL int32_t *p_out = a.p ? gmem(a.p) : nullptr;
    E *Pv = reinterpret_cast<E *>(a.scratch + (int64_t)blockIdx.x * a.scratch_bytes);
    FW_GLOBAL E *P = gmem(Pv);
    FW_GLOBAL int32_t *D = gmem(a.d + el.mat_off);
    if ((el.flags & EF_ZERO_D) && !a.closure_only) {  // no voters: d = 0
        for (int64_t i = tid; i < (int64_t)m * m; i += BT) D[i] = 0;
        __syncthreads();
    }

    // edge weights into the padded scratch matrix, 64 x 64 tiles through LDS;
    // candidates with gone[x] >= 0 (removed for top-k) lose all their edges
    int32_t *ta = reinterpret_cast<int32_t *>(smem);  // [64][65]
    int32_t *tb = ta + 64 * 65;                       // [64][65]
    int32_t *bb = tb + 64 * 65;                       // [SCHULZE_BATCH_MAX_M]
    int32_t *lvl = bb + SCHULZE_BATCH_MAX_M;          // [SCHULZE_BATCH_MAX_M]
    const int32_t nt = (mp + 63) / 64;
    auto weights = [&](const int32_t *gone) {
        bool too_big = false;
        for (int32_t I = 0; I < nt; ++I) {
            for (int32_t J = 0; J < nt; ++J) {
                __syncthreads();
                // all 32 loads in flight at once: addresses clamped into the matrix
                // (a conditional load would wait for the ones before it)
                constexpr int PER = 64 * 64 / BT;
                int32_t va[PER], vb[PER];
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int q = tid + k * BT;
                    const int r = q >> 6, c = q & 63;
                    const int32_t i = min(I * 64 + r, m - 1), j = min(J * 64 + c, m - 1);
                    const int32_t i2 = min(J * 64 + r, m - 1), j2 = min(I * 64 + c, m - 1);
                    va[k] = D[(int64_t)i * m + j];
                    vb[k] = D[(int64_t)i2 * m + j2];
                }
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int q = tid + k * BT;
                    const int r = q >> 6, c = q & 63;
                    const bool in_a = I * 64 + r < m && J * 64 + c < m;
                    const bool in_b = J * 64 + r < m && I * 64 + c < m;
                    ta[r * 65 + c] = in_a ? va[k] : 0;
                    tb[r * 65 + c] = in_b ? vb[k] : 0;
                }
                __syncthreads();
                for (int q = tid; q < 64 * 64; q += BT) {
                    const int r = q >> 6, c = q & 63;
                    const int32_t i = I * 64 + r, j = J * 64 + c;
                    if (i >= mp || j >= mp) continue;
                    const int32_t x = ta[r * 65 + c], y = tb[c * 65 + r];  // d[i][j], d[j][i]
                    int32_t w = 0;
                    if (i != j && i < m && j < m && x > y) w = mode == SCHULZE_MARGIN ? x - y : x;
                    if (gone && w && (gone[i] >= 0 || gone[j] >= 0)) w = 0;
                    if constexpr (sizeof(E) == 2) {
                        if ((uint32_t)w > 65535u) {  // counts above the bound the plan assumed
                            too_big = true;
                            w = 65535;
                        }
                    }
                    P[(int64_t)i * mp + j] = (E)w;
                }
            }
        }
        if (too_big) set_device_error(a.err, SCHULZE_ERANGE);
        __syncthreads();
    };
    // bb[x] = #{y : P[y][x] > P[x][y]}
    auto beaten = [&]() {
        for (int32_t x = tid; x < m; x += BT) bb[x] = 0;
        const int32_t mt = (m + 63) / 64;
        for (int32_t I = 0; I < mt; ++I) {      // block of x
            for (int32_t J = 0; J < mt; ++J) {  // block of y
                __syncthreads();
                constexpr int PER = 64 * 64 / BT;
                int32_t va[PER], vb[PER];
#pragma unroll
                for (int k = 0; k < PER; ++k) {  // clamped, unconditional loads
                    const int q = tid + k * BT;
                    const int r = q >> 6, c = q & 63;
                    const int32_t y = min(J * 64 + r, m - 1), x = min(I * 64 + c, m - 1);    // ta[y][x] = P[y][x]
                    const int32_t x2 = min(I * 64 + r, m - 1), y2 = min(J * 64 + c, m - 1);  // tb[x][y] = P[x][y]
                    va[k] = (int32_t)P[(int64_t)y * mp + x];
                    vb[k] = (int32_t)P[(int64_t)x2 * mp + y2];
                }
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int q = tid + k * BT;
                    const int r = q >> 6, c = q & 63;
                    ta[r * 65 + c] = (J * 64 + r < m && I * 64 + c < m) ? va[k] : 0;
                    tb[r * 65 + c] = (I * 64 + r < m && J * 64 + c < m) ? vb[k] : 0;
                }
                __syncthreads();
                const int32_t xl = tid & 63, g = tid >> 6;
                const int32_t x = I * 64 + xl;
                int32_t cnt = 0;
                for (int32_t yl = g; yl < 64; yl += 4) cnt += ta[yl * 65 + xl] > tb[xl * 65 + yl] ? 1 : 0;
                if (x < m && cnt) atomicAdd(&bb[x], cnt);
            }
        }
        __syncthreads();
    };

    weights(nullptr);
    closure_dispatch<E>(Pv, mp, el.variant);
    __syncthreads();
    beaten();

    __shared__ int32_t sh_wins;
    if (tid == 0) sh_wins = 0;
    __syncthreads();
    int32_t wins = 0;
    for (int32_t x = tid; x < m; x += BT) {
        const int32_t bx = bb[x];
        const bool win = bx == 0;
        wins += win ? 1 : 0;
        is_winner[el.vec_off + x] = win ? 1 : 0;
        if (beaten_by) beaten_by[el.vec_off + x] = bx;
        if (order) {
            int32_t rank = 0;
            for (int32_t y = 0; y < m; ++y) {
                const int32_t by = bb[y];
                rank += (by < bx || (by == bx && y < x)) ? 1 : 0;
            }
            order[el.vec_off + rank] = x;
        }
    }
    if (wins) atomicAdd(&sh_wins, wins);
    if (p_out) {
        // eight rows at a time, their loads (clamped) before their stores
        FW_GLOBAL int32_t *Pout = p_out + el.mat_off;
        constexpr int R = 8, H = SCHULZE_BATCH_MAX_M / BT;
        for (int32_t x0 = 0; x0 < m; x0 += R) {
            int32_t v[R][H];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int h = 0; h < H; ++h)
                    v[r][h] = (int32_t)P[(int64_t)min(x0 + r, m - 1) * mp + min(tid + h * BT, m - 1)];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int32_t x = x0 + r, y = tid + h * BT;
                    if (x < m && y < m) Pout[(int64_t)x * m + y] = x == y ? 0 : v[r][h];
                }
        }
    }
    __syncthreads();
    if (tid == 0 && a.n_winners) gmem(a.n_winners)[e] = sh_wins;

    // top-k by iterated winner removal: level 0 = the winners; each further
    // level closes the weights with the ranked candidates' edges deleted and
    // takes the winners among the candidates left
    if (a.level && a.topk > 0) {
        __shared__ int32_t sh_ranked, sh_new;
        for (int32_t x = tid; x < m; x += BT) lvl[x] = bb[x] == 0 ? 0 : -1;
        if (tid == 0) sh_ranked = sh_wins;
        __syncthreads();
        // every nonempty set of candidates has a winner, so each level ranks at least one
        for (int32_t level = 1; level < m && sh_ranked < a.topk && sh_ranked < m; ++level) {
            weights(lvl);
            closure_dispatch<E>(Pv, mp, el.variant);
            __syncthreads();
            beaten();
            if (tid == 0) sh_new = 0;
            __syncthreads();
            int32_t got = 0;
            for (int32_t x = tid; x < m; x += BT)
                if (lvl[x] < 0 && bb[x] == 0) {  // removed candidates have no edges: skip them
                    lvl[x] = level;
                    ++got;
                }
            if (got) atomicAdd(&sh_new, got);
            __syncthreads();
            if (tid == 0) sh_ranked += sh_new;
            __syncthreads();
        }
        FW_GLOBAL int32_t *lv = gmem(a.level);
        for (int32_t x = tid; x < m; x += BT) lv[el.vec_off + x] = lvl[x];
    }
    __syncthreads();
}

__device__ __attribute__((noinline)) void finish(const BatchArgs &a, const BElec &el_in, int32_t e) {
    const BElec el = el_in;  // local copy (see scan_item)
    if (el.flags & EF_VAL16)
        finish_t<uint16_t>(a, el, e, batch_smem);
    else
        finish_t<int32_t>(a, el, e, batch_smem);
}

__global__ __launch_bounds__(BT, 2) void k_batch(BatchArgs a) {
    __shared__ int32_t sh_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            FW_GLOBAL int32_t *ctr = gmem(a.ctr);
            int32_t t = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) t = a.n_items;
            sh_item = t;
        }
        __syncthreads();
        const int32_t t = sh_item;
        if (t >= a.n_items) return;
        const BItem it = a.items[t];
        const BElec el = a.elec[it.e];
        if (it.kind == IT_SCAN) {
            if (a.dtype32)
                scan_item<int32_t>(a, el, it.a, it.b);
            else
                scan_item<uint16_t>(a, el, it.a, it.b);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(gmem(a.ctr) + 2 + it.e, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (it.kind == IT_COUNT) {
            count_item(a, el, it.e, it.a, it.b);
        } else {
            finish(a, el, it.e);
        }
    }
}

// Pseudo-random tournament counts for timing the closure schedules:
// d[x][y] + d[y][x] = n for x != y, d[x][x] = 0.
__global__ __launch_bounds__(256) void k_tune_counts(int32_t *d, int32_t E, int32_t m, int32_t n) {
    const int64_t total = (int64_t)E * m * m;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int64_t e = q / ((int64_t)m * m);
        const int32_t r = (int32_t)(q % ((int64_t)m * m));
        const int32_t x = r / m, y = r % m;
        const int32_t lo = min(x, y), hi = max(x, y);
        uint64_t h = ((uint64_t)e << 40) ^ ((uint64_t)lo << 20) ^ (uint64_t)hi;
        h = (h ^ (h >> 30)) * 0xbf58476d1ce4e5b9ull;
        h = (h ^ (h >> 27)) * 0x94d049bb133111ebull;
        h ^= h >> 31;
        const int32_t v = (int32_t)(h % (uint64_t)(n + 1));
        d[q] = x == y ? 0 : (x < y ? v : n - v);
    }
}

}  // namespace

// ====================================================================== host

struct schulze_batch {
    schulze_ctx *ctx = nullptr;
    int device = 0;
    int32_t E = 0;
    int ballot_dtype = SCHULZE_U16;
    int mode = SCHULZE_WINNING_VOTES;
    bool closure_only = false;
    int32_t topk = 0;
    std::vector<BElec> elec;
    BElec *elec_dev = nullptr;
    BItem *items_full = nullptr, *items_closure = nullptr;
    int32_t n_full = 0, n_closure = 0;
    uint32_t *pos = nullptr;
    char *scratch = nullptr;
    int64_t scratch_bytes = 0;
    int32_t grid = 0;
    int32_t *ctr = nullptr;
    // captured graph
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchArgs key{};
};

namespace {

int default_variant(int bits, int32_t m) {
    (void)bits;
    return m <= 128 ? SCHULZE_BATCH_CLOSURE_REGISTERS : SCHULZE_BATCH_CLOSURE_TILED64;
}

bool variant_ok(int bits, int32_t m, int variant) {
    switch (variant) {
        // register budget of one workgroup at two workgroups per CU
        case SCHULZE_BATCH_CLOSURE_REGISTERS: return round_up(m, 32) <= (bits == 16 ? 192 : 128);
        case SCHULZE_BATCH_CLOSURE_TILED32: return bits == 16;
        case SCHULZE_BATCH_CLOSURE_TILED64: return true;
        case SCHULZE_BATCH_CLOSURE_TILED128: return bits == 16;
        default: return false;
    }
}

int resolve_variant(const schulze_ctx *ctx, int bits, int32_t m) {
    const int b = (int)((m - 1) / 32);
    const int v = ctx->batch_variant[bits == 16 ? 0 : 1][b];
    if (v >= 0 && variant_ok(bits, m, v)) return v;
    return default_variant(bits, m);
}

int32_t padded_size(int variant, int32_t m) {
    switch (variant) {
        case SCHULZE_BATCH_CLOSURE_REGISTERS: return (int32_t)round_up(m, 32);
        case SCHULZE_BATCH_CLOSURE_TILED32: return (int32_t)round_up(m, 32);
        case SCHULZE_BATCH_CLOSURE_TILED64: return (int32_t)round_up(m, 64);
        default: return (int32_t)round_up(m, 128);
    }
}

int batch_grid(schulze_ctx *ctx, int32_t *grid) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, BT, 0) != hipSuccess || per_cu < 1)
        return SCHULZE_EDEVICE;
    *grid = per_cu * ctx->num_cus;
    return SCHULZE_OK;
}

void free_plan(schulze_batch *pl) {
    if (!pl) return;
    (void)hipSetDevice(pl->device);
    (void)hipDeviceSynchronize();
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    for (void *ptr : {(void *)pl->elec_dev, (void *)pl->items_full, (void *)pl->items_closure, (void *)pl->pos,
                      (void *)pl->scratch, (void *)pl->ctr})
        if (ptr) (void)hipFree(ptr);
    delete pl;
}

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
    if (src.empty()) return SCHULZE_OK;
    if (hipMalloc((void **)dst, sizeof(T) * src.size()) != hipSuccess) return SCHULZE_ENOMEM;
    if (hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
        return SCHULZE_EDEVICE;
    return SCHULZE_OK;
}

int build_plan(schulze_ctx *ctx, const schulze_election *desc, int32_t E, int ballot_dtype, int mode,
               const schulze_batch_options *opt, int forced_variant, schulze_batch **out) {
    *out = nullptr;
    int32_t max_range = SEG_PAIRS;
    bool closure_only = false;
    if (opt) {
        if (opt->max_range_pairs < 0) return SCHULZE_EINVAL;
        if (opt->max_range_pairs > 0) max_range = std::min(max_range, opt->max_range_pairs);
        closure_only = opt->closure_only != 0;
        if (opt->topk < 0) return SCHULZE_EINVAL;
    }
    schulze_batch *pl = new (std::nothrow) schulze_batch();
    if (!pl) return SCHULZE_ENOMEM;
    pl->ctx = ctx;
    pl->device = ctx->device;
    pl->E = E;
    pl->ballot_dtype = ballot_dtype;
    pl->mode = mode;
    pl->closure_only = closure_only;
    pl->topk = opt ? opt->topk : 0;
    pl->elec.resize(E);
    std::vector<double> cost(E);
    std::vector<int32_t> runs_of(E), ranges_of(E);
    int64_t pos_words = 0;
    int64_t scratch = 256;
    for (int32_t e = 0; e < E; ++e) {
        const schulze_election &s = desc[e];
        BElec &el = pl->elec[e];
        el = BElec{};
        el.ballot_off = s.ballot_off;
        el.n = s.n;
        el.mat_off = s.mat_off;
        el.vec_off = s.vec_off;
        el.m = s.m;
        el.L = s.L;
        el.nb8 = (int32_t)ceil_div(s.m, 8);
        el.pitch = 8 * el.nb8;
        const bool square = s.L < s.m - 1;
        const bool val16 = s.n <= 65535;
        const int bits = val16 ? 16 : 32;
        el.variant = forced_variant >= 0 ? forced_variant : resolve_variant(ctx, bits, s.m);
        if (!variant_ok(bits, s.m, el.variant)) {
            delete pl;
            return SCHULZE_EINVAL;
        }
        el.mp = padded_size(el.variant, s.m);
        const int64_t pairs = (s.n + 1) / 2;
        const int32_t S = square ? el.nb8 * el.nb8 : el.nb8 * (el.nb8 + 1) / 2;
        el.vs = S <= 64 ? 4 : (S <= 128 ? 2 : 1);
        const int32_t runs = (int32_t)ceil_div(S, BT / el.vs);
        const int32_t nq = el.pitch / 4;
        const int32_t groups = (int32_t)ceil_div(nq, 64);
        el.ng = groups <= 1 ? 1 : (groups <= 2 ? 2 : 4);
        el.vc = 4 * MAX_PF / el.ng;
        el.range_pairs = max_range;
        const int64_t ranges = pairs > 0 ? ceil_div(pairs, max_range) : 0;
        el.flags = (square ? EF_SQUARE : 0) | (ranges > 1 ? EF_MULTI : 0) | (val16 ? EF_VAL16 : 0) |
                   (s.n == 0 ? EF_ZERO_D : 0);
        el.n_count = (int32_t)(runs * ranges);
        runs_of[e] = runs;
        ranges_of[e] = (int32_t)ranges;
        const int32_t vpb = scan_group_pairs(el.pitch);
        el.scan_pairs = (int32_t)std::max<int64_t>(vpb, std::min<int64_t>(pairs, SCAN_WORDS / el.pitch));
        el.n_scan = pairs > 0 ? (int32_t)ceil_div(pairs, el.scan_pairs) : 0;
        el.pos_off = pos_words;
        if (!closure_only) pos_words += pairs * el.pitch;
        const int64_t es = val16 ? 2 : 4;
        scratch = std::max<int64_t>(scratch, round_up(es * el.mp * el.mp, 256));
        cost[e] = closure_only ? (double)el.mp * el.mp * el.mp
                               : (double)pairs * S * 128.0 + 4.0 * (double)el.mp * el.mp * el.mp;
    }
    // queue: largest elections first
    std::vector<int32_t> order(E);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    int rc = batch_grid(ctx, &pl->grid);
    std::vector<BItem> full, fin;
    if (!closure_only && rc == SCHULZE_OK) {
        // Scans (memory-bound) run ahead of the counts (VALU-bound) by `ahead`
        // elections, so that the two overlap; every scan of an election still
        // precedes its counts in the queue.
        auto push_scans = [&](int32_t e) {
            const BElec &el = pl->elec[e];
            const int64_t pairs = (el.n + 1) / 2;
            for (int64_t q = 0; q < pairs; q += el.scan_pairs)
                full.push_back(BItem{IT_SCAN, e, (int32_t)q, (int32_t)std::min<int64_t>(el.scan_pairs, pairs - q)});
        };
        int32_t ahead = 0;
        for (int64_t items = 0; ahead < E && items < 2 * (int64_t)pl->grid; ++ahead) items += pl->elec[order[ahead]].n_count;
        for (int32_t i = 0; i < ahead; ++i) push_scans(order[i]);
        for (int32_t i = 0; i < E; ++i) {
            const int32_t e = order[i];
            for (int32_t r = 0; r < ranges_of[e]; ++r)
                for (int32_t u = 0; u < runs_of[e]; ++u) full.push_back(BItem{IT_COUNT, e, u, r});
            if (i + ahead < E) push_scans(order[i + ahead]);
        }
        for (int32_t e : order)
            if (pl->elec[e].n_count == 0) full.push_back(BItem{IT_FINISH, e, 0, 0});
    }
    for (int32_t e : order) fin.push_back(BItem{IT_FINISH, e, 0, 0});
    pl->n_full = (int32_t)full.size();
    pl->n_closure = (int32_t)fin.size();

    if (rc == SCHULZE_OK) rc = upload(&pl->elec_dev, pl->elec);
    if (rc == SCHULZE_OK) rc = upload(&pl->items_full, full);
    if (rc == SCHULZE_OK) rc = upload(&pl->items_closure, fin);
    if (rc == SCHULZE_OK && pos_words > 0 &&
        hipMalloc((void **)&pl->pos, sizeof(uint32_t) * (size_t)pos_words) != hipSuccess)
        rc = SCHULZE_ENOMEM;
    pl->scratch_bytes = scratch;
    if (rc == SCHULZE_OK && hipMalloc((void **)&pl->scratch, (size_t)scratch * pl->grid) != hipSuccess)
        rc = SCHULZE_ENOMEM;
    if (rc == SCHULZE_OK && hipMalloc((void **)&pl->ctr, sizeof(int32_t) * (size_t)(2 + 2 * (int64_t)E)) != hipSuccess)
        rc = SCHULZE_ENOMEM;
    if (rc != SCHULZE_OK) {
        (void)hipGetLastError();
        free_plan(pl);
        return rc;
    }
    *out = pl;
    return SCHULZE_OK;
}

// The reset of the counters and the persistent launch (graph-capturable).
int enqueue(schulze_batch *pl, hipStream_t s, const BatchArgs &args) {
    schulze_ctx *ctx = pl->ctx;
    int rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(pl->ctr), (size_t)(2 + 2 * (int64_t)pl->E), 0u);
    if (rc != SCHULZE_OK) return rc;
    if (args.n_items == 0) return SCHULZE_OK;
    SCHULZE_LAUNCH(ctx, K_BATCH, s, k_batch<<<dim3((unsigned)pl->grid), dim3(BT), 0, s>>>(args));
    return SCHULZE_OK;
}

bool same_args(const BatchArgs &x, const BatchArgs &y) {
    return x.ballots == y.ballots && x.d == y.d && x.p == y.p && x.is_winner == y.is_winner &&
           x.n_winners == y.n_winners && x.beaten_by == y.beaten_by && x.order == y.order &&
           x.level == y.level && x.topk == y.topk && x.closure_only == y.closure_only && x.err == y.err;
}

}  // namespace

extern "C" int schulze_batch_plan(schulze_ctx *ctx, const schulze_election *elections, int32_t E, int ballot_dtype,
                                  int mode, const schulze_batch_options *opt, schulze_batch **plan) {
    if (!plan) return SCHULZE_EINVAL;
    *plan = nullptr;
    if (!ctx || E < 0 || (E > 0 && !elections)) return SCHULZE_EINVAL;
    if (ballot_dtype != SCHULZE_U16 && ballot_dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (mode != SCHULZE_WINNING_VOTES && mode != SCHULZE_MARGIN) return SCHULZE_EINVAL;
    if (E > (1 << 24)) return SCHULZE_EUNSUPPORTED;
    for (int32_t e = 0; e < E; ++e) {
        const schulze_election &s = elections[e];
        if (s.m < 1 || s.m > SCHULZE_BATCH_MAX_M || s.L < 1 || s.L > s.m || s.n < 0) return SCHULZE_EINVAL;
        if (s.ballot_off < 0 || s.mat_off < 0 || s.vec_off < 0) return SCHULZE_EINVAL;
        if (s.n > (int64_t)INT32_MAX) return SCHULZE_EUNSUPPORTED;
    }
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    return build_plan(ctx, elections, E, ballot_dtype, mode, opt, -1, plan);
}

extern "C" void schulze_batch_destroy(schulze_batch *plan) { free_plan(plan); }

extern "C" int schulze_batch_run(schulze_ctx *ctx, void *stream, schulze_batch *plan, const void *ballots, int32_t *d,
                                 int32_t *p, uint8_t *is_winner, int32_t *n_winners, int32_t *beaten_by,
                                 int32_t *order, int32_t *level, int flags) {
    if (!ctx || !plan || plan->ctx != ctx || !d || !is_winner) return SCHULZE_EINVAL;
    if (level && plan->topk == 0) return SCHULZE_EINVAL;
    if (flags & ~SCHULZE_BATCH_GRAPH) return SCHULZE_EINVAL;
    const bool closure_only = ballots == nullptr;
    if (!closure_only && plan->closure_only) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    BatchArgs args{};
    args.elec = plan->elec_dev;
    args.items = closure_only ? plan->items_closure : plan->items_full;
    args.n_items = closure_only ? plan->n_closure : plan->n_full;
    args.n_elec = plan->E;
    args.ballots = ballots;
    args.dtype32 = plan->ballot_dtype == SCHULZE_I32;
    args.mode = plan->mode;
    args.closure_only = closure_only ? 1 : 0;
    args.pos = plan->pos;
    args.d = d;
    args.p = p;
    args.is_winner = is_winner;
    args.n_winners = n_winners;
    args.beaten_by = beaten_by;
    args.order = order;
    args.level = level;
    args.topk = level ? plan->topk : 0;
    args.ctr = plan->ctr;
    args.scratch = plan->scratch;
    args.scratch_bytes = plan->scratch_bytes;
    args.err = ctx->err;
    if (!(flags & SCHULZE_BATCH_GRAPH)) return enqueue(plan, s, args);

    if (!plan->exec || !same_args(plan->key, args)) {
        if (plan->exec) {
            (void)hipGraphExecDestroy(plan->exec);
            plan->exec = nullptr;
        }
        if (plan->graph) {
            (void)hipGraphDestroy(plan->graph);
            plan->graph = nullptr;
        }
        if (!plan->cap && hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking) != hipSuccess)
            return SCHULZE_EDEVICE;
        if (hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return SCHULZE_EDEVICE;
        const bool timing = ctx->timing;
        ctx->timing = false;
        int rc = enqueue(plan, plan->cap, args);
        ctx->timing = timing;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(plan->cap, &g);
        if (rc != SCHULZE_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return rc != SCHULZE_OK ? rc : SCHULZE_EDEVICE;
        }
        if (hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            plan->exec = nullptr;
            return SCHULZE_EDEVICE;
        }
        plan->graph = g;
        plan->key = args;
    }
    int tok;
    timing_begin(ctx, K_BATCH, s, &tok);
    const hipError_t e = hipGraphLaunch(plan->exec, s);
    timing_end(ctx, tok, s);
    return e == hipSuccess ? SCHULZE_OK : SCHULZE_EDEVICE;
}

extern "C" int schulze_batch_set_closure(schulze_ctx *ctx, int32_t value_bits, int32_t m_lo, int32_t m_hi,
                                         int32_t variant) {
    if (!ctx || (value_bits != 16 && value_bits != 32)) return SCHULZE_EINVAL;
    if (m_lo < 1 || m_hi < m_lo || m_hi > SCHULZE_BATCH_MAX_M) return SCHULZE_EINVAL;
    if (variant < SCHULZE_BATCH_CLOSURE_AUTO || variant > SCHULZE_BATCH_CLOSURE_TILED128) return SCHULZE_EINVAL;
    for (int32_t m = m_lo; m <= m_hi; ++m)
        if (variant >= 0 && !variant_ok(value_bits, m, variant)) return SCHULZE_EINVAL;
    for (int32_t b = (m_lo - 1) / 32; b <= (m_hi - 1) / 32; ++b)
        ctx->batch_variant[value_bits == 16 ? 0 : 1][b] = (int8_t)variant;
    return SCHULZE_OK;
}

extern "C" int schulze_batch_get_closure(schulze_ctx *ctx, int32_t value_bits, int32_t m, int32_t *variant) {
    if (!ctx || !variant || (value_bits != 16 && value_bits != 32) || m < 1 || m > SCHULZE_BATCH_MAX_M)
        return SCHULZE_EINVAL;
    *variant = resolve_variant(ctx, value_bits, m);
    return SCHULZE_OK;
}

extern "C" int schulze_batch_autotune(schulze_ctx *ctx, void *stream, int32_t value_bits, int32_t m_max,
                                      float *ms) {
    if (!ctx || (value_bits != 16 && value_bits != 32) || m_max < 1 || m_max > SCHULZE_BATCH_MAX_M)
        return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    int32_t grid = 0;
    int rc = batch_grid(ctx, &grid);
    if (rc != SCHULZE_OK) return rc;
    const int32_t nbk = (int32_t)ceil_div(m_max, 32);
    const int32_t m_top = nbk * 32;
    const int32_t E = grid;  // one election per resident workgroup
    const int32_t n = value_bits == 16 ? 60000 : 1000000;
    int32_t *d = nullptr;
    uint8_t *win = nullptr;
    if (hipMalloc((void **)&d, sizeof(int32_t) * (size_t)E * m_top * m_top) != hipSuccess) return SCHULZE_ENOMEM;
    if (hipMalloc((void **)&win, (size_t)E * m_top) != hipSuccess) {
        (void)hipFree(d);
        return SCHULZE_ENOMEM;
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) rc = SCHULZE_EDEVICE;
    const bool timing = ctx->timing;
    ctx->timing = false;
    for (int32_t b = 0; b < nbk && rc == SCHULZE_OK; ++b) {
        const int32_t m = 32 * (b + 1);
        k_tune_counts<<<dim3((unsigned)ctx->num_cus * 4), dim3(256), 0, s>>>(d, E, m, n);
        if ((rc = launch_status()) != SCHULZE_OK) break;
        std::vector<schulze_election> desc(E);
        for (int32_t e = 0; e < E; ++e)
            desc[e] = schulze_election{0, n, m, m, (int64_t)e * m * m, (int64_t)e * m};
        schulze_batch_options opt{};
        opt.closure_only = 1;
        float best = 0.f;
        int best_v = -1;
        for (int v = SCHULZE_BATCH_CLOSURE_REGISTERS; v <= SCHULZE_BATCH_CLOSURE_TILED128 && rc == SCHULZE_OK; ++v) {
            if (ms) ms[b * 4 + v] = -1.f;
            if (!variant_ok(value_bits, m, v)) continue;
            schulze_batch *pl = nullptr;
            if ((rc = build_plan(ctx, desc.data(), E, SCHULZE_U16, SCHULZE_WINNING_VOTES, &opt, v, &pl)) !=
                SCHULZE_OK)
                break;
            float t = 0.f;
            rc = schulze_batch_run(ctx, stream, pl, nullptr, d, nullptr, win, nullptr, nullptr, nullptr, nullptr, 0);
            for (int rep = 0; rep < 2 && rc == SCHULZE_OK; ++rep) {
                float tr = 0.f;
                if (hipEventRecord(t0, s) != hipSuccess) rc = SCHULZE_EDEVICE;
                if (rc == SCHULZE_OK)
                    rc = schulze_batch_run(ctx, stream, pl, nullptr, d, nullptr, win, nullptr, nullptr, nullptr, nullptr, 0);
                if (rc == SCHULZE_OK &&
                    (hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                     hipEventElapsedTime(&tr, t0, t1) != hipSuccess))
                    rc = SCHULZE_EDEVICE;
                t = rep == 0 ? tr : std::min(t, tr);
            }
            free_plan(pl);
            if (rc != SCHULZE_OK) break;
            if (ms) ms[b * 4 + v] = t;
            if (best_v < 0 || t < best) {
                best = t;
                best_v = v;
            }
        }
        if (rc == SCHULZE_OK && best_v >= 0) ctx->batch_variant[value_bits == 16 ? 0 : 1][b] = (int8_t)best_v;
    }
    ctx->timing = timing;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(d);
    (void)hipFree(win);
    return rc;
}
