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
// All three are exact in integers, so the result does not depend on B or on
// the order in which independent tiles are processed.
//
// Main path: one persistent launch.  Every tile has a fixed owner workgroup
// (its state never leaves that workgroup's XCD).  An owner publishes the
// round-r diagonal and panel tiles into a write-once buffer (one slot per
// round and tile) and raises a flag; consumers wait on the flags they need.
// Each workgroup works through its tiles round by round with a lookahead of
// one round: panels of round r, then (for its owner) tile (r+1, r+1) and at
// once round r+1's diagonal, then the other tiles that feed round r+1, then
// round r+1's panels if that diagonal is out already, then the other rest
// tiles of round r.  Round r+1 thus starts while round r is still running.
// Order the items diag(0), panels(0), diag(1), panels(1), ...: a workgroup
// only waits for an item earlier in that order than every item it has yet to
// publish, and a cooperative launch keeps all workgroups resident, so every
// wait ends;
// a bounded spin turns anything else into a device error instead of a hang.
//
// uint16 matrices run two columns per 32-bit lane with v_pk_min_u16 and
// v_pk_max_u16 (one instruction per update); int32 matrices use v_min_i32
// and v_max3_i32 over pairs of k.  The matrix is padded with zero rows and
// columns to a multiple of B; padded vertices have no edges and change
// nothing.
#include "fw_tiles.h"
#include "tile_io.h"


namespace {

using namespace fw;

// A launch can be gated on a device word: it runs only when *gate == want
// (gate == nullptr: always).  The int32 closure decides on the device
// whether its values can be ranked, and both variants are queued with
// opposite gates, so the host never waits for the decision.
__device__ inline bool gated_off(const int32_t *gate, int32_t want) { return gate && *gate != want; }

// ------------------------------------------------------------------ weights
// P[i][j] = edge weight from d (winning votes or margin); zero padding.  A
// workgroup takes the pair of 64 x 64 tiles (I, J) and (J, I), I <= J: both
// need the same two blocks of d, so every count is read once.
template <typename E>
__global__ __launch_bounds__(256) void k_weights(const E *__restrict__ d, int64_t ldd, int32_t m, int mode,
                                                 E *__restrict__ P, int64_t ld, int32_t mp, int dvec,
                                                 const int32_t *gate = nullptr, int32_t want = 0) {
    __shared__ E a[64][65];  // a[r][c] = d[I0 + r][J0 + c]
    __shared__ E b[64][65];  // b[r][c] = d[J0 + r][I0 + c]
    if (blockIdx.y > blockIdx.x || gated_off(gate, want)) return;
    const int32_t I0 = blockIdx.y * 64, J0 = blockIdx.x * 64;
    tio::load<E>(a, d, ldd, I0, J0, m, m, dvec != 0);
    tio::load<E>(b, d, ldd, J0, I0, m, m, dvec != 0);
    __syncthreads();
    auto weight = [&](E x, E y, bool diag) -> E {  // edge weight given d[i][j] = x, d[j][i] = y
        if (diag || x <= y) return (E)0;
        return mode == SCHULZE_MARGIN ? (E)(x - y) : x;
    };
    // the workspace matrix is 16-byte aligned with a pitch that is a multiple of 64
    tio::store<E>(P, ld, I0, J0, mp, mp, true, [&](int r, int c) { return weight(a[r][c], b[c][r], I0 + r == J0 + c); });
    if (I0 != J0)  // the mirrored tile (J, I)
        tio::store<E>(P, ld, J0, I0, mp, mp, true, [&](int r, int c) { return weight(b[r][c], a[c][r], false); });
}

// p[i][j] = P[i][j] for i != j, 0 on the diagonal; one workgroup per row.
template <typename E>
__global__ __launch_bounds__(256) void k_fw_store(const E *__restrict__ P, int64_t ld, int32_t m, E *__restrict__ p,
                                                  int64_t ldp, const int32_t *gate, int32_t want) {
    if (gated_off(gate, want)) return;
    const int32_t i = blockIdx.x;
    const E *src = P + (int64_t)i * ld;
    E *dst = p + (int64_t)i * ldp;
    for (int32_t j = threadIdx.x; j < m; j += 256) dst[j] = i == j ? (E)0 : src[j];
}

// ------------------------------------------------------------------ persistent launch
template <typename E>
struct PersistArgs {
    E *P;               // padded matrix, pitch ld
    int64_t ld;
    int32_t nb;
    E *ring;            // nb rounds x (2 nb + 1) published tiles of B x B
    int32_t *flags;     // nb x (2 nb + 1), zero on entry
    int32_t *abort;     // zero on entry
    int32_t *err;       // device error word
    int64_t spin_limit; // polls before a wait is declared stuck
    int32_t early_panels; // run round r+1's panels ahead of round r's last tiles when possible
    const int32_t *gate;  // run only if *gate == gate_want (nullptr: always)
    int32_t gate_want;
};

constexpr int MAX_OWNED = 512;

// Owner of tile (I, J): tile (I, J) is number I nb + (I + J) mod nb (block
// rows in order, each rotated by its index) and the numbers are dealt to the
// G workgroups in turn.  Every workgroup owns floor or ceil of nb^2 / G
// tiles (all of them take part whatever nb is), a block row spreads over
// distinct workgroups when nb <= G, and a block column too when G is a
// multiple of nb, so that the panels of a round are computed in parallel.
// (32-bit arithmetic: the host launches the kernel only for nb^2 <= MAX_OWNED G)
__device__ inline int32_t tile_owner(int32_t I, int32_t J, int32_t nb, int32_t G) {
    return (int32_t)(((uint32_t)I * (uint32_t)nb + (uint32_t)((I + J) % nb)) % (uint32_t)G);
}

// slot of a published tile within a round: 0 diag, 1+J row panel, 1+nb+I column panel
__device__ inline int64_t slot_index(int32_t r, int32_t slot, int32_t nb) { return (int64_t)r * (2 * nb + 1) + slot; }

__device__ inline bool wait_flags(const int32_t *f0, const int32_t *f1, int32_t *abort, int64_t limit) {
    __shared__ int32_t ok;
    if (threadIdx.x == 0) {
        int32_t good = 1;
        int64_t spins = 0;
        const int32_t *fs[2] = {f0, f1};
        for (int q = 0; q < 2 && good; ++q) {
            if (!fs[q]) continue;
            while (__hip_atomic_load(fs[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > limit) {
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        ok = good;
    }
    __syncthreads();
    const bool res = ok != 0;
    __syncthreads();
    return res;
}

// Whether a flag is raised already (no waiting); uniform over the workgroup.
__device__ inline bool probe_flag(const int32_t *f) {
    __shared__ int32_t seen;
    if (threadIdx.x == 0) seen = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const bool res = seen != 0;
    __syncthreads();
    return res;
}

// Raise the flag of a published tile once this workgroup's stores of it are
// visible device-wide.  Published slots are written with agent-scope stores
// (they do not stay in this XCD's L2), so it suffices that every thread's
// stores have been acknowledged (vmcnt 0) before the barrier and the flag
// store; an agent-scope release fence would also write back every dirty line
// of the L2, which takes microseconds on the critical path.  Tiles of P are
// only ever read by their owner within the launch.  Published slots are
// written once per launch and read only after their flag is seen, so no
// reader can hold an older copy of them.
constexpr int16_t WAIT_VMCNT0 = 0x0F70;  // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15) (gfx9 encoding)
__device__ inline void raise_flag(int32_t *f) {
    __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// acc_store with stores coherent at agent scope (not held in this XCD's L2),
// for the published tiles.
template <typename E, int B>
__device__ inline void acc_store_agent(const Acc<E, B> &a, E *dst, int64_t ld) {
    using C = Cfg<E, B>;
    const int t = lane_tid(), tx = t & 15, ty = t >> 4;
    dst = scalar_ptr(dst);
    for (int ii = 0; ii < C::TM; ++ii) {
        uint32_t *row = reinterpret_cast<uint32_t *>(dst + (int64_t)(ty * C::TM + ii) * ld + tx * C::TN);
        for (int jj = 0; jj < C::WN; ++jj)
            __hip_atomic_store(row + jj, __builtin_bit_cast(uint32_t, a.c[ii][jj]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename E, int B>
__global__ __launch_bounds__(256, sizeof(E) == 2 ? 4 : (B < 128 ? 2 : 1)) void k_fw_persist(PersistArgs<E> a) {
    using C = Cfg<E, B>;
    constexpr int DS = diag_steps<E, B>();
    constexpr int DIAG_LDS = diag_lds_elems<E, B, DS, true>();
    __shared__ __attribute__((aligned(16))) E lds[C::LDS_ELEMS > DIAG_LDS ? C::LDS_ELEMS : DIAG_LDS];
    __shared__ int32_t owned[MAX_OWNED];
    __shared__ int32_t n_owned;
    const int32_t nb = a.nb, G = gridDim.x, w = blockIdx.x;
    const int64_t tile_elems = (int64_t)B * B;
    if (gated_off(a.gate, a.gate_want)) return;  // uniform over the grid: every workgroup leaves

    // Tiles this workgroup owns, in ascending tile number: the numbers
    // k = w, w + G, w + 2G, ... stand for block row I = k / nb and column
    // J = (k mod nb - I) mod nb (the inverse of the owner map below).
    if (threadIdx.x == 0) n_owned = (int32_t)((nb * nb - w + G - 1) / G);
    __syncthreads();
    const int32_t no = n_owned;
    for (int32_t q = threadIdx.x; q < no && q < MAX_OWNED; q += 256) {
        const int32_t k = w + q * G, I = k / nb;
        owned[q] = I * nb + ((k % nb) - I + nb) % nb;
    }
    __syncthreads();
    if (no > MAX_OWNED) {  // the host sizes the grid so that this cannot happen
        if (threadIdx.x == 0) {
            set_device_error(a.err, SCHULZE_EDEVICE);
            __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }

    // owned[q] through a scalar register: tile numbers are uniform, and
    // everything derived from them (tile addresses, flags) then stays in
    // scalar registers rather than taking vector ones
    auto tile_at = [&](int32_t q) { return __builtin_amdgcn_readfirstlane(owned[q]); };
    auto tileP = [&](int32_t I, int32_t J) { return a.P + (int64_t)I * B * a.ld + (int64_t)J * B; };
    auto ring = [&](int32_t r, int32_t slot) { return a.ring + slot_index(r, slot, nb) * tile_elems; };
    auto flag = [&](int32_t r, int32_t slot) { return a.flags + slot_index(r, slot, nb); };

    // One panel of round r (a tile of block row or column r, updated in place
    // and published).
    auto do_panel = [&](int32_t r, int32_t I, int32_t J) {
        Acc<E, B> acc;
        acc_load<E, B>(acc, tileP(I, J), a.ld);
        int32_t slot;
        if (I == r) {  // row panel: D* (x) P[r][J]
            acc_product<E, B>(acc, ring(r, 0), B, tileP(I, J), a.ld, lds);
            slot = 1 + J;
        } else {       // column panel: P[I][r] (x) D*
            acc_product<E, B>(acc, tileP(I, J), a.ld, ring(r, 0), B, lds);
            slot = 1 + nb + I;
        }
        acc_store<E, B>(acc, tileP(I, J), a.ld);
        acc_store_agent<E, B>(acc, ring(r, slot), B);
        raise_flag(flag(r, slot));
    };
    // A rest tile of round r.  When `probe` is given, thread 0 also reads
    // that flag (issued before the product, so its latency hides behind the
    // tile) and the workgroup learns whether it was raised.
    __shared__ int32_t probe_seen;
    auto do_rest = [&](int32_t r, int32_t I, int32_t J, const int32_t *probe) -> bool {
        if (!wait_flags(flag(r, 1 + J), flag(r, 1 + nb + I), a.abort, a.spin_limit)) return false;
        int32_t seen = 0;
        if (probe && threadIdx.x == 0) seen = __hip_atomic_load(probe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Acc<E, B> acc;
        acc_load<E, B>(acc, tileP(I, J), a.ld);
        acc_product<E, B>(acc, ring(r, 1 + nb + I), B, ring(r, 1 + J), B, lds);
        acc_store<E, B>(acc, tileP(I, J), a.ld);
        if (probe) {
            if (threadIdx.x == 0) probe_seen = seen;
            __syncthreads();
        }
        return true;
    };
    auto has_panels = [&](int32_t r) {
        for (int32_t q = 0; q < no; ++q) {
            const int32_t t_ = tile_at(q), I = t_ / nb, J = t_ % nb;
            if ((I == r) != (J == r)) return true;
        }
        return false;
    };
    // All of this workgroup's panels of round r (its diagonal is published).
    // Panels gate every rest tile of their round, so their waves take the
    // SIMDs first.
    auto run_panels = [&](int32_t r) {
        __builtin_amdgcn_s_setprio(3);
        for (int32_t q = 0; q < no; ++q) {
            const int32_t t_ = tile_at(q), I = t_ / nb, J = t_ % nb;
            if ((I == r) == (J == r)) continue;
            do_panel(r, I, J);
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // Lookahead.  Round r+1 can start as soon as its diagonal tile has its
    // round-r update, so the owner of tile (r+1, r+1) updates it first and
    // closes it at once, and the owners of the other tiles of block row and
    // column r+1 update those next.  The chain diagonal -> panels next to it
    // -> next diagonal is the critical path of the recurrence: its tiles run
    // at raised wave priority, and the owner of a panel that feeds the next
    // diagonal waits for its diagonal and computes it right away.  Other
    // workgroups, with early_panels, look at the round-(r+1) diagonal flag
    // while they run their remaining round-r tiles and compute their
    // round-(r+1) panels as soon as it is up, so that round r+1's tiles find
    // their panels ready.
    // (Round -1 only closes diagonal tile 0.)
    int32_t panels_done = -1;  // round whose panels this workgroup already ran
    int32_t diag_done = -1;    // last diagonal tile this workgroup closed
    for (int32_t r = -1; r < nb; ++r) {
        if (r >= 0 && panels_done != r) {
            if (has_panels(r)) {
                if (!wait_flags(flag(r, 0), nullptr, a.abort, a.spin_limit)) goto stuck;
                run_panels(r);
            }
            panels_done = r;
        }
        bool next_panels = false;  // round r+1's panels are still to do
        if (r + 1 < nb) {
            // the next diagonal tile
            if (tile_owner(r + 1, r + 1, nb, G) == w && diag_done < r + 1) {
                __builtin_amdgcn_s_setprio(3);
                if (r >= 0 && !do_rest(r, r + 1, r + 1, nullptr)) goto stuck;
                diag_close<E, B, DS, true>(tileP(r + 1, r + 1), a.ld, tileP(r + 1, r + 1), a.ld, ring(r + 1, 0), B,
                                           lds);
                raise_flag(flag(r + 1, 0));
                __builtin_amdgcn_s_setprio(0);
                diag_done = r + 1;
            }
            if (r < 0) continue;
            // the other tiles that feed round r+1
            for (int32_t q = 0; q < no; ++q) {
                const int32_t t_ = tile_at(q), I = t_ / nb, J = t_ % nb;
                if (I == r || J == r || (I != r + 1 && J != r + 1) || (I == r + 1 && J == r + 1)) continue;
                if (!do_rest(r, I, J, nullptr)) goto stuck;
            }
            next_panels = a.early_panels && has_panels(r + 1);
            const bool critical = r + 2 < nb && (tile_owner(r + 1, r + 2, nb, G) == w ||
                                                 tile_owner(r + 2, r + 1, nb, G) == w);
            if (next_panels && (critical || probe_flag(flag(r + 1, 0)))) {
                if (!wait_flags(flag(r + 1, 0), nullptr, a.abort, a.spin_limit)) goto stuck;
                run_panels(r + 1);
                panels_done = r + 1;
                next_panels = false;
            }
        }
        // Two rounds ahead: the owner of tile (r+2, r+2) gives it its
        // round-r update now, waits for the round-(r+1) panels next to it
        // and closes it as round r+2's diagonal, instead of reaching it
        // after its other round-r tiles.
        int32_t ahead = -1;
        if (a.early_panels && nb <= G && r + 2 < nb && tile_owner(r + 2, r + 2, nb, G) == w) {
            __builtin_amdgcn_s_setprio(3);
            if (!do_rest(r, r + 2, r + 2, nullptr)) goto stuck;
            if (!do_rest(r + 1, r + 2, r + 2, nullptr)) goto stuck;
            diag_close<E, B, DS, true>(tileP(r + 2, r + 2), a.ld, tileP(r + 2, r + 2), a.ld, ring(r + 2, 0), B, lds);
            raise_flag(flag(r + 2, 0));
            __builtin_amdgcn_s_setprio(0);
            diag_done = r + 2;
            ahead = (r + 2) * nb + (r + 2);
        }
        // the remaining rest tiles of round r
        if (threadIdx.x == 0) probe_seen = 0;
        __syncthreads();
        for (int32_t q = 0; q < no; ++q) {
            const int32_t t_ = tile_at(q), I = t_ / nb, J = t_ % nb;
            if (I == r || J == r || I == r + 1 || J == r + 1 || t_ == ahead) continue;
            if (next_panels && probe_seen) {  // (uniform: written before a barrier)
                run_panels(r + 1);
                panels_done = r + 1;
                next_panels = false;
            }
            if (!do_rest(r, I, J, next_panels ? flag(r + 1, 0) : nullptr)) goto stuck;
        }
    }
    return;
stuck:
    if (threadIdx.x == 0) set_device_error(a.err, SCHULZE_EDEVICE);
}

// ------------------------------------------------------------------ per-phase launches
// Used when a cooperative launch is not available: three launches per round.
template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_diag(E *__restrict__ P, int64_t ld, int32_t r, const int32_t *gate,
                                                 int32_t want) {
    if (gated_off(gate, want)) return;
    __shared__ __attribute__((aligned(16))) E buf[diag_lds_elems<E, B, diag_steps<E, B>(), true>()];
    E *t = P + (int64_t)r * B * ld + (int64_t)r * B;
    diag_close<E, B, diag_steps<E, B>(), true>(t, ld, t, ld, nullptr, 0, buf);
}

template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_panel(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r,
                                                  const int32_t *gate, int32_t want) {
    if (gated_off(gate, want)) return;
    __shared__ __attribute__((aligned(16))) E lds[Cfg<E, B>::LDS_ELEMS];
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
    E *Ct = P + (int64_t)I * B * ld + (int64_t)J * B;
    Acc<E, B> acc;
    acc_load<E, B>(acc, Ct, ld);
    acc_product<E, B>(acc, P + (int64_t)I * B * ld + (int64_t)r * B, ld, P + (int64_t)r * B * ld + (int64_t)J * B,
                      ld, lds);
    acc_store<E, B>(acc, Ct, ld);
}

template <typename E, int B>
__global__ __launch_bounds__(256) void k_fw_rest(E *__restrict__ P, int64_t ld, int32_t nb, int32_t r,
                                                 const int32_t *gate, int32_t want) {
    if (gated_off(gate, want)) return;
    __shared__ __attribute__((aligned(16))) E lds[Cfg<E, B>::LDS_ELEMS];
    const int32_t t = blockIdx.x;
    const int32_t i = t / (nb - 1), j = t % (nb - 1);
    const int32_t I = i < r ? i : i + 1, J = j < r ? j : j + 1;
    E *Ct = P + (int64_t)I * B * ld + (int64_t)J * B;
    Acc<E, B> acc;
    acc_load<E, B>(acc, Ct, ld);
    acc_product<E, B>(acc, P + (int64_t)I * B * ld + (int64_t)r * B, ld, P + (int64_t)r * B * ld + (int64_t)J * B,
                      ld, lds);
    acc_store<E, B>(acc, Ct, ld);
}

// Device memory of the persistent launch: published tiles and their flags.
template <typename E, int B>
size_t ring_bytes(int32_t nb) {
    return sizeof(E) * (size_t)nb * (2 * (size_t)nb + 1) * B * B;
}
inline size_t flag_bytes(int32_t nb) { return sizeof(int32_t) * ((size_t)nb * (2 * (size_t)nb + 1) + 64); }

// Launch the persistent kernel.  Outside stream capture it is a cooperative
// launch (all workgroups resident).  Under capture it is captured as a
// cooperative launch when the runtime allows; otherwise as a plain launch of
// the same occupancy-sized grid, whose workgroups are all resident whenever
// the device is not running other work, and whose bounded waits report
// SCHULZE_EDEVICE instead of hanging if they ever are not.
inline hipError_t launch_persistent(const void *fn, unsigned G, void **args, hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(256), args, 0, s);
    if (e == hipSuccess || cap != hipStreamCaptureStatusActive) return e;
    (void)hipGetLastError();
    hipStreamCaptureStatus now = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &now) != hipSuccess || now != hipStreamCaptureStatusActive) return e;
    return hipLaunchKernel(fn, dim3(G), dim3(256), args, 0, s);
}

// Close the padded matrix P (pitch ld, nb x nb tiles of B) in place: one
// persistent dataflow launch, or three launches per round when the device
// refuses a cooperative launch or the phased schedule is forced.  Every
// launch is gated on (gate, want) (see gated_off).
template <typename E, int B>
int close_padded(schulze_ctx *ctx, hipStream_t s, E *P, int64_t ld, int32_t nb, const int32_t *gate = nullptr,
                 int32_t want = 0) {
    int rc;
    bool done = false;
    if (nb > 1 && !ctx->force_phased) {
        // persistent dataflow launch
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fw_persist<E, B>, 256, 0) != hipSuccess)
            per_cu = 0;
        int64_t G = (int64_t)per_cu * ctx->num_cus;
        if (G > (int64_t)nb * nb) G = (int64_t)nb * nb;
        const int64_t tiles_per_wg = ceil_div((int64_t)nb * nb, G > 0 ? G : 1);
        if (G >= 1 && tiles_per_wg <= MAX_OWNED) {
            const int64_t nslots = (int64_t)nb * (2 * nb + 1);
            if ((rc = ws_reserve(ctx, WS_RING, ring_bytes<E, B>(nb))) != SCHULZE_OK) return rc;
            if ((rc = ws_reserve(ctx, WS_FLAGS, flag_bytes(nb))) != SCHULZE_OK) return rc;
            int32_t *flags = static_cast<int32_t *>(ctx->ws[WS_FLAGS]);
            if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(flags), (size_t)(nslots + 64), 0u)) != SCHULZE_OK)
                return rc;
            // early panels and the two-rounds-ahead diagonal while each workgroup
            // has few tiles per round: at most 20 (uint16) or 8 (int32); measured
            // on one MI355X: uint16 m = 12288 66.1 -> 62.1 ms, m = 14187 112.8 ->
            // 111.6 ms, m = 16384 146.4 -> 148 ms (hence off there)
            const int32_t early = (int64_t)nb * nb <= (sizeof(E) == 2 ? 20 : 8) * G ? 1 : 0;
            PersistArgs<E> pa{P,     ld,    nb, static_cast<E *>(ctx->ws[WS_RING]), flags, flags + nslots, ctx->err,
                              (int64_t)1 << 22, early, gate, want};
            void *args[] = {&pa};
            int tok;
            timing_begin(ctx, K_FW_PERSIST, s, &tok);
            hipError_t e = launch_persistent((const void *)k_fw_persist<E, B>, (unsigned)G, args, s);
            timing_end(ctx, tok, s);
            if (e == hipSuccess) {
                done = true;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    if (!done) {
        for (int32_t r = 0; r < nb; ++r) {
            SCHULZE_LAUNCH(ctx, K_FW_DIAG, s, k_fw_diag<E, B><<<dim3(1), dim3(256), 0, s>>>(P, ld, r, gate, want));
            if (nb > 1) {
                SCHULZE_LAUNCH(ctx, K_FW_PANEL, s,
                               k_fw_panel<E, B><<<dim3((unsigned)(2 * (nb - 1))), dim3(256), 0, s>>>(P, ld, nb, r,
                                                                                                     gate, want));
                SCHULZE_LAUNCH(ctx, K_FW_REST, s,
                               k_fw_rest<E, B><<<dim3((unsigned)((nb - 1) * (nb - 1))), dim3(256), 0, s>>>(
                                   P, ld, nb, r, gate, want));
            }
        }
    }
    return SCHULZE_OK;
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
    SCHULZE_LAUNCH(ctx, K_WEIGHTS, s, k_weights<E><<<wgrid, dim3(256), 0, s>>>(d, ldd, m, mode, P, ld, mp,
                                                                          tio::vec_ok<E>(d, ldd) ? 1 : 0));
    if ((rc = close_padded<E, B>(ctx, s, P, ld, nb)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_FW_STORE, s,
                   k_fw_store<E><<<dim3((unsigned)m), dim3(256), 0, s>>>(P, ld, m, p, ldp, nullptr, 0));
    ctx->closure_bits = sizeof(E) * 8;
    return SCHULZE_OK;
}

// ------------------------------------------------------------------ ranked int32 closures
// The (max, min) recurrence commutes with every strictly increasing map of
// the values (the max and min of mapped values are the mapped max and min),
// and such a map can fix 0.  So when the int32 weights take at most 65535
// distinct nonzero values, all below RANK_CAP, the closure runs on their
// ranks (1 = smallest nonzero value) in packed uint16 -- one instruction per
// update instead of one and a half -- and the result is mapped back through
// the table of ranked values.  Exact; otherwise the int32 closure runs.
constexpr int32_t RANK_CAP = 1 << 24;           // values ranked below this bound
constexpr int32_t RANK_WORDS = RANK_CAP / 32;   // bitmap words
constexpr int32_t RANK_BLOCK = 1024;            // bitmap words per scan block
constexpr int32_t RANK_BLOCKS = RANK_WORDS / RANK_BLOCK;
constexpr int32_t RANK_MIN_M = 1024;            // below this the decision's synchronisation is not worth it

// Values below RANK_LDS_BITS (the frequent small ones) are gathered in a
// workgroup bitmap in LDS and merged once per workgroup, so that the global
// bitmap sees one atomic per set word and workgroup instead of one per
// repeated value.
constexpr int32_t RANK_LDS_WORDS = 1024;  // 4 KB: values below 2^15 (with the two tiles, four workgroups per CU;
                                          // 32 KB and two per CU took 0.60 ms at m = 16384, this 0.45 ms)
constexpr int32_t RANK_LDS_BITS = RANK_LDS_WORDS * 32;

// Per block of RANK_BLOCK words: number of marked values.
__global__ __launch_bounds__(256) void k_rank_blocks(const uint32_t *__restrict__ bitmap,
                                                     uint32_t *__restrict__ block_sum) {
    __shared__ uint32_t part[256];
    const uint32_t *w = bitmap + (int64_t)blockIdx.x * RANK_BLOCK;
    uint32_t c = 0;
    for (int i = threadIdx.x; i < RANK_BLOCK; i += 256) c += __popc(w[i]);
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sum[blockIdx.x] = part[0];
}

// Exclusive scan of the block sums (one workgroup); flags[1] = number of
// distinct nonzero values; flags[2] = 1 if the closure runs on ranks (no
// value at or above RANK_CAP, at most 65535 distinct values), else 0.
__global__ __launch_bounds__(256) void k_rank_top(uint32_t *__restrict__ block_sum, int32_t *__restrict__ flags) {
    __shared__ uint32_t part[256];
    constexpr int PER = RANK_BLOCKS / 256;
    uint32_t v[PER];
    uint32_t c = 0;
    for (int i = 0; i < PER; ++i) {
        v[i] = block_sum[threadIdx.x * PER + i];
        c += v[i];
    }
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scan
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - c;
    for (int i = 0; i < PER; ++i) {
        block_sum[threadIdx.x * PER + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 255) {
        flags[1] = (int32_t)part[255];
        flags[2] = (flags[0] == 0 && part[255] <= 65535u) ? 1 : 0;
    }
}

// word_rank[w] = number of marked values below word w; value_of[r] = the
// value of rank r (1-based) while r <= 65535.
__global__ __launch_bounds__(256) void k_rank_words(const uint32_t *__restrict__ bitmap,
                                                    const uint32_t *__restrict__ block_off,
                                                    uint32_t *__restrict__ word_rank, int32_t *__restrict__ value_of,
                                                    const int32_t *gate) {
    if (gated_off(gate, 1)) return;
    __shared__ uint32_t part[256];
    constexpr int PER = RANK_BLOCK / 256;
    const int64_t w0 = (int64_t)blockIdx.x * RANK_BLOCK + threadIdx.x * PER;
    uint32_t words[PER], c = 0;
    for (int i = 0; i < PER; ++i) {
        words[i] = bitmap[w0 + i];
        c += __popc(words[i]);
    }
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = block_off[blockIdx.x] + part[threadIdx.x] - c;
    for (int i = 0; i < PER; ++i) {
        word_rank[w0 + i] = run;
        uint32_t bits = words[i];
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1;
            ++run;
            if (run <= 65535u) value_of[run] = (int32_t)((w0 + i) * 32 + b);
        }
    }
}

// Edge weight from d[i][j] = x and d[j][i] = y (0 on the diagonal and where
// x <= y), as in k_weights.
__device__ inline int32_t weight_of(int32_t x, int32_t y, bool diag, int mode) {
    if (diag || x <= y) return 0;
    return mode == SCHULZE_MARGIN ? x - y : x;
}

// (I, J), I <= J, of pair q in the order J = 0, 1, ... and I = 0..J.
__device__ inline void pair_of(int64_t q, int32_t &I, int32_t &J) {
    int64_t j = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > q) --j;
    while ((j + 1) * (j + 2) / 2 <= q) ++j;
    J = (int32_t)j;
    I = (int32_t)(q - j * (j + 1) / 2);
}

// Every nonzero weight value marked in the bitmap (flags[0] = 1 if a value
// is >= RANK_CAP), straight from d: the weights of both tiles of each pair
// of 64 x 64 blocks (I, J), (J, I) are computed as in k_weights and never
// written (the ranked closure needs only their ranks; the int32 closure, if
// the values cannot be ranked, writes its own weights).  Persistent over the
// pairs, so that each workgroup merges its LDS bitmap once; the next pair's
// tiles are loaded into registers while the current pair is marked (VEC:
// 16-byte loads, d 16-byte aligned with m a multiple of 4; what they read
// past m is ignored).
template <bool VEC>
__global__ __launch_bounds__(256) void k_weights_mark(const int32_t *__restrict__ d, int64_t ldd, int32_t m,
                                                      int mode, uint32_t *__restrict__ bitmap,
                                                      int32_t *__restrict__ flags) {
    __shared__ int32_t a[64][65];  // a[r][c] = d[I0 + r][J0 + c]
    __shared__ int32_t b[64][65];  // b[r][c] = d[J0 + r][I0 + c]
    __shared__ uint32_t local[RANK_LDS_WORDS];
    for (int i = threadIdx.x; i < RANK_LDS_WORDS; i += 256) local[i] = 0u;
    bool wide = false;
    auto mark = [&](int32_t v) {
        if (v == 0) return;
        if (v >= RANK_CAP || v < 0) {
            wide = true;
            return;
        }
        const uint32_t bit = 1u << (v & 31);
        if (v < RANK_LDS_BITS) {
            if (!(local[v >> 5] & bit)) atomicOr(&local[v >> 5], bit);
        } else {
            uint32_t *word = bitmap + (v >> 5);
            if (!(*word & bit)) atomicOr(word, bit);
        }
    };
    const int32_t nt = (m + 63) / 64;
    const int64_t npairs = (int64_t)nt * (nt + 1) / 2;
    tio::Regs<int32_t> ga, gb;
    auto fetch_pair = [&](int64_t q) {
        int32_t I, J;
        pair_of(q, I, J);
        tio::fetch<int32_t, VEC>(ga, d, ldd, I * 64, J * 64, m, m);
        tio::fetch<int32_t, VEC>(gb, d, ldd, J * 64, I * 64, m, m);
    };
    if (blockIdx.x < npairs) fetch_pair(blockIdx.x);
    for (int64_t q = blockIdx.x; q < npairs; q += gridDim.x) {
        int32_t I, J;
        pair_of(q, I, J);
        const int32_t I0 = I * 64, J0 = J * 64;
        __syncthreads();  // the previous pair's tiles are read
        tio::put<int32_t>(a, ga);
        tio::put<int32_t>(b, gb);
        __syncthreads();
        if (q + gridDim.x < npairs) fetch_pair(q + gridDim.x);
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            // (each tile's own bounds: a partial tile's rows are the other's columns)
            if (I0 + r < m && J0 + c < m) mark(weight_of(a[r][c], b[c][r], I0 + r == J0 + c, mode));
            if (I != J && J0 + r < m && I0 + c < m) mark(weight_of(b[r][c], a[c][r], false, mode));
        }
    }
    if (wide) flags[0] = 1;
    __syncthreads();
    for (int i = threadIdx.x; i < RANK_LDS_WORDS; i += 256)
        if (local[i]) atomicOr(&bitmap[i], local[i]);
}

// P16 = rank of the weights of d (0 for 0), straight from d: one workgroup
// per pair of 64 x 64 blocks (I, J), (J, I) of the padded mp x mp matrix
// (zero past m); the table lookups of a thread's 32 elements are issued
// together before the ranks are formed.
__global__ __launch_bounds__(256) void k_rank_apply_d(const int32_t *__restrict__ d, int64_t ldd, int32_t m,
                                                      int mode, int dvec, const uint32_t *__restrict__ bitmap,
                                                      const uint32_t *__restrict__ word_rank,
                                                      uint16_t *__restrict__ P16, int64_t ld, int32_t mp,
                                                      const int32_t *gate) {
    __shared__ int32_t a[64][65];
    __shared__ int32_t b[64][65];
    if (blockIdx.y > blockIdx.x || gated_off(gate, 1)) return;
    const int32_t I0 = blockIdx.y * 64, J0 = blockIdx.x * 64;
    tio::load<int32_t>(a, d, ldd, I0, J0, m, m, dvec != 0);
    tio::load<int32_t>(b, d, ldd, J0, I0, m, m, dvec != 0);
    __syncthreads();
    // thread: rows r = t / 8 and r + 32, eight columns from c8 = 8 (t % 8); both tiles
    const int r0 = threadIdx.x >> 3, c8 = (threadIdx.x & 7) * 8;
    int32_t w[2][2][8];  // [tile][row][column]
    for (int h = 0; h < 2; ++h)
        for (int u = 0; u < 8; ++u) {
            const int r = r0 + 32 * h, c = c8 + u;
            w[0][h][u] = weight_of(a[r][c], b[c][r], I0 + r == J0 + c, mode);
            w[1][h][u] = I0 != J0 ? weight_of(b[r][c], a[c][r], false, mode) : 0;
        }
    uint32_t bw[2][2][8], wr[2][2][8];
    for (int t = 0; t < 2; ++t)
        for (int h = 0; h < 2; ++h)
            for (int u = 0; u < 8; ++u) {
                const uint32_t wd = (uint32_t)w[t][h][u] >> 5;  // values are below RANK_CAP when this runs
                bw[t][h][u] = bitmap[wd];
                wr[t][h][u] = word_rank[wd];
            }
    for (int t = 0; t < 2; ++t) {
        if (t == 1 && I0 == J0) break;
        const int32_t R0 = t ? J0 : I0, C0 = t ? I0 : J0;
        for (int h = 0; h < 2; ++h) {
            const int32_t row = R0 + r0 + 32 * h;
            if (row >= mp) continue;
            uint16_t k[8];
            for (int u = 0; u < 8; ++u) {
                const int32_t v = w[t][h][u];
                k[u] = v == 0 ? (uint16_t)0
                              : (uint16_t)(wr[t][h][u] + __popc(bw[t][h][u] & ((1u << (v & 31)) - 1u)) + 1u);
            }
            // mp and ld are multiples of 64 and P16 is 16-byte aligned: eight columns are one store
            *reinterpret_cast<uint4 *>(P16 + (int64_t)row * ld + C0 + c8) = tio::pack<uint16_t>(k);
        }
    }
}

// p[i][j] = value_of[P16[i][j]] for i != j, 0 on the diagonal; one
// workgroup per row, four columns per thread and step (ld is a multiple of 64).
__global__ __launch_bounds__(256) void k_rank_store(const uint16_t *__restrict__ P16, int64_t ld, int32_t m,
                                                    const int32_t *__restrict__ value_of, int32_t *__restrict__ p,
                                                    int64_t ldp, const int32_t *gate) {
    if (gated_off(gate, 1)) return;
    const int32_t i = blockIdx.x;
    int32_t *row = p + (int64_t)i * ldp;
    // STORE_STEP groups of four columns per thread and step; every load and
    // table lookup unconditional (P16 rows hold ld >= m columns, a multiple
    // of 64; rank 0 looks up value_of[0] = 0), the stores under the bounds
    constexpr int STORE_STEP = 4;
    const bool vec = (ldp % 4) == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0;
    for (int32_t jb = threadIdx.x * 4; jb < m; jb += 1024 * STORE_STEP) {
        ushort4 r[STORE_STEP];
        for (int u = 0; u < STORE_STEP; ++u)
            r[u] = *reinterpret_cast<const ushort4 *>(P16 + (int64_t)i * ld + min(jb + 1024 * u, (int32_t)ld - 4));
        int32_t v[STORE_STEP][4];
        for (int u = 0; u < STORE_STEP; ++u) {
            v[u][0] = value_of[r[u].x];
            v[u][1] = value_of[r[u].y];
            v[u][2] = value_of[r[u].z];
            v[u][3] = value_of[r[u].w];
        }
        for (int u = 0; u < STORE_STEP; ++u) {
            const int32_t j0 = jb + 1024 * u;
            if (j0 >= m) break;
            for (int e = 0; e < 4; ++e)
                if (j0 + e == i) v[u][e] = 0;
            if (vec && j0 + 4 <= m)
                *reinterpret_cast<int4 *>(row + j0) = make_int4(v[u][0], v[u][1], v[u][2], v[u][3]);
            else
                for (int e = 0; e < 4 && j0 + e < m; ++e) row[j0 + e] = v[u][e];
        }
    }
}

// BI: tile of the int32 closure (when the values cannot be ranked); BU: tile
// of the uint16 closure on the ranks.
template <int BI, int BU>
int run_closure_ranked(schulze_ctx *ctx, hipStream_t s, const int32_t *d, int64_t ldd, int32_t m, int mode, int32_t *p,
                       int64_t ldp) {
    constexpr int B = BI > BU ? BI : BU;
    static_assert(B % BI == 0 && B % BU == 0, "both tiles divide the padded size");
    const int32_t mp = (int32_t)round_up(m, B);
    const int64_t ld = mp;
    const int64_t count = (int64_t)mp * mp;
    // rank tables: bitmap | word ranks | block offsets | value table | flags, then the uint16 matrix
    const size_t bm = sizeof(uint32_t) * RANK_WORDS;
    const size_t bo = sizeof(uint32_t) * RANK_BLOCKS;
    const size_t vt = sizeof(int32_t) * 65536;
    const size_t head = 2 * bm + bo + vt + 256;
    // all workspace up front, for both variants: nothing grows (and so
    // nothing synchronises) once work is queued
    int rc = ws_reserve(ctx, WS_CLOSURE, sizeof(int32_t) * (size_t)count);
    if (rc != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_RANKED, head + sizeof(uint16_t) * (size_t)count)) != SCHULZE_OK) return rc;
    if ((rc = ws_reserve(ctx, WS_RING, std::max(ring_bytes<int32_t, BI>(mp / BI), ring_bytes<uint16_t, BU>(mp / BU)))) !=
        SCHULZE_OK)
        return rc;
    if ((rc = ws_reserve(ctx, WS_FLAGS, std::max(flag_bytes(mp / BI), flag_bytes(mp / BU)))) != SCHULZE_OK) return rc;
    int32_t *P = static_cast<int32_t *>(ctx->ws[WS_CLOSURE]);
    const int dvec = tio::vec_ok<int32_t>(d, ldd) ? 1 : 0;

    char *q = static_cast<char *>(ctx->ws[WS_RANKED]);
    uint32_t *bitmap = reinterpret_cast<uint32_t *>(q);
    uint32_t *word_rank = reinterpret_cast<uint32_t *>(q + bm);
    uint32_t *block_off = reinterpret_cast<uint32_t *>(q + 2 * bm);
    int32_t *value_of = reinterpret_cast<int32_t *>(q + 2 * bm + bo);
    int32_t *flags = reinterpret_cast<int32_t *>(q + 2 * bm + bo + vt);
    uint16_t *P16 = reinterpret_cast<uint16_t *>(q + head);
    if ((rc = fill_u32(ctx, s, bitmap, RANK_WORDS, 0u)) != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(value_of), 1, 0u)) != SCHULZE_OK) return rc;
    if ((rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(flags), 3, 0u)) != SCHULZE_OK) return rc;
    // The weights' values are marked straight from d (the weights are not
    // written here): four marking workgroups per CU, each merging its LDS
    // bitmap once.
    const unsigned mgrid = (unsigned)std::min<int64_t>(ceil_div((int64_t)m * m, 8192), (int64_t)ctx->num_cus * 4);
    if (dvec && m % 4 == 0)
        SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                       k_weights_mark<true><<<dim3(mgrid), dim3(256), 0, s>>>(d, ldd, m, mode, bitmap, flags));
    else
        SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                       k_weights_mark<false><<<dim3(mgrid), dim3(256), 0, s>>>(d, ldd, m, mode, bitmap, flags));
    SCHULZE_LAUNCH(ctx, K_RANK, s, k_rank_blocks<<<dim3(RANK_BLOCKS), dim3(256), 0, s>>>(bitmap, block_off));
    SCHULZE_LAUNCH(ctx, K_RANK, s, k_rank_top<<<dim3(1), dim3(256), 0, s>>>(block_off, flags));
    // flags[2] decides on the device; both variants are queued, each gated
    const int32_t *ranked = flags + 2;
    const dim3 wgrid((unsigned)ceil_div(mp, 64), (unsigned)ceil_div(mp, 64));
    // values too wide or too many: the weights, then the int32 closure on them
    SCHULZE_LAUNCH(ctx, K_WEIGHTS, s,
                   k_weights<int32_t><<<wgrid, dim3(256), 0, s>>>(d, ldd, m, mode, P, ld, mp, dvec, ranked, 0));
    if ((rc = close_padded<int32_t, BI>(ctx, s, P, ld, mp / BI, ranked, 0)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_FW_STORE, s,
                   k_fw_store<int32_t><<<dim3((unsigned)m), dim3(256), 0, s>>>(P, ld, m, p, ldp, ranked, 0));
    // otherwise the ranks of the weights (straight from d) and the uint16 closure on them
    SCHULZE_LAUNCH(ctx, K_RANK, s,
                   k_rank_words<<<dim3(RANK_BLOCKS), dim3(256), 0, s>>>(bitmap, block_off, word_rank, value_of,
                                                                        ranked));
    SCHULZE_LAUNCH(ctx, K_RANK, s,
                   k_rank_apply_d<<<wgrid, dim3(256), 0, s>>>(d, ldd, m, mode, dvec, bitmap, word_rank, P16, ld, mp,
                                                              ranked));
    if ((rc = close_padded<uint16_t, BU>(ctx, s, P16, ld, mp / BU, ranked, 1)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_RANK, s,
                   k_rank_store<<<dim3((unsigned)m), dim3(256), 0, s>>>(P16, ld, m, value_of, p, ldp, ranked));
    ctx->closure_bits = 0;
    ctx->closure_ranked_flag = ranked;
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
    const int tile = ctx->closure_tile;
    const int bu = tile ? tile : (m >= 6144 ? 128 : 64);  // uint16 tile
    const int bi = tile ? tile : (m >= 2048 ? 128 : 64);  // int32 tile
    const int32_t *di = static_cast<const int32_t *>(d);
    int32_t *pi = static_cast<int32_t *>(p);
    if (dtype == SCHULZE_U16)
        return bu == 128 ? run_closure<uint16_t, 128>(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode,
                                                      static_cast<uint16_t *>(p), ldp)
                         : run_closure<uint16_t, 64>(ctx, s, static_cast<const uint16_t *>(d), ldd, m, mode,
                                                     static_cast<uint16_t *>(p), ldp);
    if (m >= RANK_MIN_M && ctx->value_ranking) {
        if (bi == 128)
            return bu == 128 ? run_closure_ranked<128, 128>(ctx, s, di, ldd, m, mode, pi, ldp)
                             : run_closure_ranked<128, 64>(ctx, s, di, ldd, m, mode, pi, ldp);
        return bu == 128 ? run_closure_ranked<64, 128>(ctx, s, di, ldd, m, mode, pi, ldp)
                         : run_closure_ranked<64, 64>(ctx, s, di, ldd, m, mode, pi, ldp);
    }
    return bi == 128 ? run_closure<int32_t, 128>(ctx, s, di, ldd, m, mode, pi, ldp)
                     : run_closure<int32_t, 64>(ctx, s, di, ldd, m, mode, pi, ldp);
}
