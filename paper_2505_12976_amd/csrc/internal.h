// Internal declarations of the Schulze GPU library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/schulze.h"

// Workspace slots owned by a context.  Each slot is a grow-only device
// buffer; a call that needs more than the slot holds reallocates it.
enum WsSlot {
    WS_BALLOT_META = 0,  // per-ballot listed length and class, counters
    WS_POSITIONS,        // packed rank pairs of full rankings
    WS_TRUNC_POS,        // packed rank pairs of truncated ballots (U space)
    WS_ACC32,            // m x m uint32 accumulator of the count
    WS_ROWSUM,           // per-candidate uint32 sums
    WS_CLOSURE,          // padded closure matrix
    WS_RANK,             // ranking keys
    WS_RING,             // closure tiles published once per round
    WS_FLAGS,            // closure publication flags
    WS_VERIFY,           // widest-path sweeps: value vectors, frontiers, barrier
    WS_FEATURES,         // per-candidate raw statistics
    WS_MLP,              // BF16 copies of the network weights
    WS_MLP_PARTIAL,      // per-workgroup gradient partials
    WS_LEARNED,          // learned path: features, scores, check outputs
    WS_LEARNED_W,        // learned path: weights of the checks after the first
    WS_LEARNED_P,        // learned path: closure for the fallback
    WS_PROPAGATE,        // label propagation: weights, keys, frontiers, statuses
    WS_RANKED,           // ranked closure: value bitmap, rank tables, uint16 matrix
    WS_OCC,              // bucketed pair counting: histograms, offsets, occurrences
    WS_MLP_TRAIN,        // train step: scores and their gradient
    WS_NUM_SLOTS
};

struct PendingTiming {
    int name;
    hipEvent_t start, stop;
};

// Polls of a frontier sweep's grid barrier before it is declared stuck.
constexpr int64_t SWEEP_SPIN_LIMIT = (int64_t)1 << 24;

struct schulze_ctx {
    int device = 0;
    int num_cus = 0;
    int32_t *err = nullptr;  // device error word
    void *ws[WS_NUM_SLOTS] = {};
    size_t ws_bytes[WS_NUM_SLOTS] = {};
    // per-kernel timing
    bool timing = false;
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<int64_t> launches;
    std::vector<double> total_ms;
    // closure schedule: false = one persistent launch when possible
    bool force_phased = false;
    // int32 closures of m >= 1024 run on value ranks in uint16 when the values allow it
    bool value_ranking = true;
    // closure tile size: 0 = by value width and m, else 64 or 128
    int closure_tile = 0;
    // value width of the last closure: 16 or 32, or 0 when the device decided
    // (then *closure_ranked_flag is 1 for ranks in uint16, 0 for int32)
    int closure_bits = 0;
    const int32_t *closure_ranked_flag = nullptr;
    // device address of schulze_verify_noalloc's static scratch on this context's device
    void *verify_scratch = nullptr;
    // first proposal of the learned path (SCHULZE_PROPOSER_*)
    int proposer = SCHULZE_PROPOSER_NETWORK;
    // limits of the frontier sweeps' bounded waits (0: the defaults), for
    // tests of their failure paths (schulze_set_sweep_limits)
    int64_t sweep_spin_limit = 0;
    int32_t sweep_max_sweeps = 0;
    // truncated ballots: pair scattering with device-wide atomics instead of bucketing
    bool legacy_pairs = false;
    // batch closure schedule per value width (16, 32) and bucket of 32 candidates; -1 = built-in
    int8_t batch_variant[2][SCHULZE_BATCH_MAX_M / 32];
    schulze_ctx() {
        for (auto &row : batch_variant)
            for (auto &v : row) v = -1;
    }
};

// Kernel names used by the timing facility (index = id).
enum KernelId {
    K_BALLOT_SCAN = 0,
    K_BALLOT_SCATTER,
    K_COUNT_DENSE,
    K_COUNT_SPARSE,
    K_COUNT_FINISH,
    K_WEIGHTS,
    K_FW_DIAG,
    K_FW_PANEL,
    K_FW_REST,
    K_FW_STORE,
    K_BEATEN_BY,
    K_RANK_SORT,
    K_WINNERS,
    K_FILL,
    K_FW_PERSIST,
    K_ROUTE,
    K_COUNT_TRUNC,
    K_WIDEST,
    K_VERDICT,
    K_FEATURES,
    K_MLP_PREP,
    K_MLP_FWD,
    K_MLP_BWD,
    K_MLP_LOSS,
    K_MLP_ADAM,
    K_PROPOSE,
    K_BATCH,
    K_PROP,
    K_PROP_SWEEP,
    K_RANK,
    K_FEATURE_ROWS,
    K_VALU_PROBE,
    K_NUM_KERNELS
};
extern const char *const kKernelNames[K_NUM_KERNELS];

// Device error word helpers (used inside kernels): the first error wins.
__device__ inline void set_device_error(int32_t *err, int32_t code) {
    atomicCAS(err, 0, code);
}

// Make sure `slot` holds at least `bytes`; returns SCHULZE_OK or ENOMEM.
int ws_reserve(schulze_ctx *ctx, WsSlot slot, size_t bytes);

// Bracket a launch with events when timing is on.
void timing_begin(schulze_ctx *ctx, int kernel, hipStream_t s, int *token);
void timing_end(schulze_ctx *ctx, int token, hipStream_t s);

// Check the last launch; returns SCHULZE_OK or SCHULZE_EDEVICE.
int launch_status();

// Zero `words` 32-bit words with a fill kernel (graph-capture friendly).
int fill_u32(schulze_ctx *ctx, hipStream_t s, uint32_t *ptr, size_t words, uint32_t value);

// Signed weights S = w - w^T of d (int32; pitch lds): both weight rules
// give a pair an edge in at most one direction, so w[i][j] = max(S[i][j], 0)
// and w[j][i] = max(-S[i][j], 0).  Arguments already checked.
int signed_weights(schulze_ctx *ctx, hipStream_t s, const int32_t *d, int64_t ldd, int32_t m, int mode, int32_t *S,
                   int64_t lds);

// schulze_verify over signed weights sw = w - w^T (int32, pitch ld);
// arguments already checked.
int verify_signed(schulze_ctx *ctx, hipStream_t s, const int32_t *sw, int64_t ld, int32_t m, int32_t cand,
                  const float *score, int32_t *p_from, int32_t *p_to, int32_t *verdict, int32_t *tied);

// Device address of the static scratch of schulze_verify_noalloc on `device`
// (looked up once per device; the device must be current).
int verify_scratch_init(int device, void **ptr);

// Bind the context's device to the calling thread.
int bind_device(schulze_ctx *ctx);

#define SCHULZE_LAUNCH(ctx, kid, stream, ...)                  \
    do {                                                        \
        int tok_;                                               \
        timing_begin((ctx), (kid), (stream), &tok_);            \
        __VA_ARGS__;                                            \
        timing_end((ctx), tok_, (stream));                      \
        int rc_ = launch_status();                              \
        if (rc_ != SCHULZE_OK) return rc_;                      \
    } while (0)

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
