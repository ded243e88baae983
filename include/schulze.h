/*
 * schulze.h -- C ABI of the MI355X (gfx950) Schulze hot-path library.
 *
 * The library computes, for one election given as a preference profile,
 * the quantities of the Schulze method as the paper defines them in its
 * voting preliminaries (Section 2.1):
 *
 *   schulze_pairwise   d[x][y] = total weight of voters who strictly prefer
 *                      candidate x to candidate y;
 *   schulze_closure    p[x][y] = width of a widest x->y path in the weighted
 *                      tournament graph built from d (width of a path = its
 *                      smallest edge weight), computed by a blocked
 *                      Floyd-Warshall over (max, min) -- the classical
 *                      algorithm the paper compares against (Section 5.2);
 *   schulze_winners    x is a Schulze winner iff no y beats x, where y beats
 *                      x iff p[y][x] > p[x][y];
 *   schulze_ranking    candidates ordered by the number of candidates that
 *                      beat them, then by id.
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers into memory the caller owns
 *    (e.g. torch tensors); the library never frees them.  The context owns
 *    only its internal workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue work on that stream and return without waiting; outputs
 *    are valid once the stream has been synchronised.
 *  - Matrices are row-major with a leading dimension (ld*) in elements,
 *    ld >= m.  Candidate ids are 0..m-1 (the paper numbers them 1..m).
 *  - Errors found on the host (bad arguments, unsupported sizes, failed
 *    allocation or launch) are returned at once as a negative code and
 *    nothing is enqueued.  Errors found in the data (an invalid ballot, a
 *    count that overflows uint16) are written to the context's device error
 *    word and reported by schulze_get_device_error.  No C++ exception
 *    crosses this boundary.
 *  - A context is not thread-safe: use one context per host thread/stream.
 */
#ifndef SCHULZE_H
#define SCHULZE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct schulze_ctx schulze_ctx;

/* Counter width of d and p.  Closure values are a subset of {0} u values(d),
 * so p fits the same type as d. */
typedef enum { SCHULZE_U16 = 1, SCHULZE_I32 = 2 } schulze_dtype;

/* Edge weight of the weighted tournament graph.
 *  WINNING_VOTES: w[x][y] = d[x][y] if d[x][y] > d[y][x], else 0.
 *  MARGIN:        w[x][y] = d[x][y] - d[y][x] if positive, else 0 -- the
 *                 majority margin mu restricted to its positive part
 *                 (Section 2.1).
 * For profiles of full strict rankings both give the same winners and
 * ranking (the margin is 2 d[x][y] - n, a strictly increasing function). */
typedef enum { SCHULZE_WINNING_VOTES = 0, SCHULZE_MARGIN = 1 } schulze_weight_mode;

enum {
    SCHULZE_OK = 0,
    SCHULZE_EINVAL = -1,       /* bad argument (null pointer, size, ld, enum) */
    SCHULZE_ERANGE = -2,       /* counts do not fit the requested dtype */
    SCHULZE_ENOMEM = -3,       /* workspace allocation failed */
    SCHULZE_EDEVICE = -4,      /* HIP runtime error (launch, copy, device) */
    SCHULZE_EBALLOT = -5,      /* ballot lists an id out of range or twice */
    SCHULZE_EUNSUPPORTED = -6  /* valid request this build does not handle */
};

/* Create a context bound to HIP device `device`.  On success *ctx is set and
 * SCHULZE_OK returned; on failure *ctx is NULL. */
int schulze_create(schulze_ctx **ctx, int device);

/* Release the context and its workspace.  Synchronises the device first.
 * NULL is accepted. */
void schulze_destroy(schulze_ctx *ctx);

/* Static string for an error code (never NULL). */
const char *schulze_strerror(int code);

/* Wait for `stream`, copy the device error word to *err_host (SCHULZE_OK if
 * no data error occurred since the last call) and reset it. */
int schulze_get_device_error(schulze_ctx *ctx, void *stream, int32_t *err_host);

/*
 * Pairwise preference counts d (Section 2.1: profile of weak orders).
 *
 * ballots       n x L candidate ids, row-major, best first.  ballot_dtype
 *               SCHULZE_U16 (uint16 ids, 0xFFFF = padding; needs m <= 65535)
 *               or SCHULZE_I32 (int32 ids, any negative = padding).  Each row
 *               lists its ranked candidates and ends at its first padding
 *               entry; candidates not listed are tied below every listed one.
 *               A row listing an id >= m or the same id twice sets the
 *               device error word to SCHULZE_EBALLOT (d is then undefined).
 * n, L, m       voters (n >= 0), row length (1 <= L <= m), candidates
 *               (1 <= m <= 65535).
 * voter_weight  NULL (every voter counts once) or n uint32 multiplicities.
 * d_dtype       SCHULZE_U16 requires the total weight to be <= 65535: with
 *               voter_weight == NULL this is checked on the host (n > 65535
 *               -> SCHULZE_ERANGE); with weights, an overflowing count sets
 *               the device error word to SCHULZE_ERANGE.  SCHULZE_I32 requires
 *               counts < 2^31 (device error SCHULZE_ERANGE otherwise).  With
 *               weights the total weight must also stay below 2^32 (counts
 *               accumulate in 32 bits); a larger total sets SCHULZE_ERANGE.
 * d, ldd        output m x m matrix, d[x][x] = 0.
 *
 * Workspace: up to m*m*4 bytes plus about n*m*2 bytes for full rankings.
 */
int schulze_pairwise(schulze_ctx *ctx, void *stream, const void *ballots, int ballot_dtype,
                     int64_t n, int32_t L, int32_t m, const uint32_t *voter_weight,
                     int d_dtype, void *d, int64_t ldd);

/*
 * Widest-path closure (Section 2.1 "widest paths"; the Floyd-Warshall
 * algorithm of Section 5.2, blocked).
 *
 * d, ldd   m x m pairwise counts (as written by schulze_pairwise), dtype.
 * mode     edge weights built from d (schulze_weight_mode).
 * p, ldp   output m x m: p[x][y] = width of a widest x->y path, 0 if y is
 *          unreachable from x; p[x][x] = 0.  p must not overlap d.
 * Exact integer arithmetic; results are independent of blocking.
 * Never waits on the host, so it can be captured in a HIP graph, provided an
 * earlier call of at least the same m and dtype has sized the context's
 * workspace (growing it synchronises the device, which capture forbids).
 */
int schulze_closure(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                    int dtype, int mode, void *p, int64_t ldp);

/*
 * Schulze winners (Section 2.1: a candidate no other candidate beats).
 *
 * p, ldp     closure from schulze_closure (dtype as given there).
 * is_winner  m bytes: 1 for winners, 0 otherwise.
 * n_winners  NULL or one device int32 receiving the number of winners
 *            (always >= 1 for a closure produced by this library).
 */
int schulze_winners(schulze_ctx *ctx, void *stream, const void *p, int64_t ldp, int32_t m,
                    int dtype, uint8_t *is_winner, int32_t *n_winners);

/*
 * Ranking (Section 2.1: the order R by p(a,b) >= p(b,a), winners on top).
 *
 * beaten_by  NULL or m int32: beaten_by[x] = number of y with p[y][x] > p[x][y].
 * order      m int32: candidates sorted by (beaten_by ascending, id ascending).
 *            Whenever a beats b, a comes before b; when R is a weak order its
 *            classes are the runs of equal beaten_by, and the first run is the
 *            winner set.
 */
int schulze_ranking(schulze_ctx *ctx, void *stream, const void *p, int64_t ldp, int32_t m,
                    int dtype, int32_t *order, int32_t *beaten_by);

/*
 * Edge weights of the weighted tournament graph (Section 2.1), the input of
 * the widest-path computations below.
 *
 * d, ldd    m x m pairwise counts; dtype as for schulze_closure.
 * mode      schulze_weight_mode.
 * w, ldw    NULL or output m x m: w[i][j] = weight of edge (i, j), 0 = no edge.
 * wt, ldwt  NULL or output m x m transposed weights: wt[j][i] = w[i][j]
 *           (the single-target direction reads it row by row).
 * At least one of w, wt must be given.
 */
int schulze_weights(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                    int dtype, int mode, void *w, int64_t ldw, void *wt, int64_t ldwt);

/*
 * Single-source widest paths: out[v] = p(source, v), the width of a widest
 * source->v path (Section 2.1), out[source] = 0.  Given transposed weights
 * it yields the single-target widths p(v, source).  Exact: (max, min)
 * relaxation sweeps over the rows whose value grew, to the fixpoint, in one
 * cooperative launch (after a plain launch that sets up the sweep state).
 * Returns SCHULZE_EDEVICE if the device refuses a cooperative launch.
 */
int schulze_widest_from(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, int32_t m,
                        int dtype, int32_t source, void *out);

/*
 * Exact winner check of one candidate, the deterministic form of the
 * NL-membership argument (Section 3): cand is a Schulze winner iff
 * p(cand, x) >= p(x, cand) for every x.
 *
 * w, wt      weights and transposed weights (schulze_weights).
 * score      NULL or m floats used to pick the reported beater.
 * p_from     m outputs: p(cand, x).     p_to: m outputs: p(x, cand).
 * verdict    4 device int32: [0] 1 if cand is a winner, [1] number of x
 *            that beat cand, [2] one beater (highest score; without scores
 *            the widest margin p(x,cand) - p(cand,x); ties -> lowest id) or
 *            -1, [3] number of x != cand tied with it (p(cand,x) = p(x,cand)).
 * tied       NULL or m device int32 receiving the tied candidates (any order).
 * Every winner is tied with every other winner, so when cand wins the
 * winner set is cand plus the tied candidates that pass the same check.
 */
int schulze_verify(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, const void *wt,
                   int64_t ldwt, int32_t m, int dtype, int32_t cand, const float *score,
                   void *p_from, void *p_to, int32_t *verdict, int32_t *tied);

/*
 * schulze_verify straight from the pairwise counts (Section 3's membership
 * argument, as above): the same outputs and verdict, but the weights are
 * formed from d inside the widest-path sweeps (w[i][j] from d[i][j] and
 * d[j][i], Section 2.1), so no weight matrix is written first.  A sweep with
 * few frontier vertices reads their rows and columns of d; one with more
 * than about m/16 relaxes every edge in one pass over d.
 *
 * d, ldd     m x m pairwise counts (dtype), device memory.
 * mode       schulze_weight_mode.
 * p_from, p_to  m elements of dtype each; verdict, tied as for schulze_verify.
 * Asynchronous on the stream; uses the context's workspace.  Returns
 * SCHULZE_EINVAL for bad arguments, SCHULZE_EUNSUPPORTED for m > 65535,
 * SCHULZE_EDEVICE if the device refuses the cooperative launch (a sweep
 * that gives up on its bounded wait sets the device error word instead).
 */
int schulze_verify_counts(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m, int dtype,
                          int mode, int32_t cand, const float *score, void *p_from, void *p_to, int32_t *verdict,
                          int32_t *tied);

/*
 * schulze_verify for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, outputs and errors as schulze_verify, but the sweep state
 * lives in a static device array of 3 MiB per device, whose address the
 * library looks up when a context is created, instead of the context's
 * workspace; the call allocates nothing.  Limit: widest-path state of both
 * directions, 32 m + 5 KB bytes, i.e. every m <= 65535 (larger m:
 * SCHULZE_EUNSUPPORTED).
 * All calls on one device share that array and leave the last call's state
 * in it: calls that overlap on one device (other streams, other contexts,
 * other host threads) race and must be serialised by the caller.
 */
int schulze_verify_noalloc(schulze_ctx *ctx, void *stream, const void *w, int64_t ldw, const void *wt,
                           int64_t ldwt, int32_t m, int dtype, int32_t cand, const float *score,
                           void *p_from, void *p_to, int32_t *verdict, int32_t *tied);

/*
 * Per-candidate features of the weighted tournament graph (the learned
 * proposer's input), computed from d in one pass:
 *   feat[x][0..15] = Copeland score, ties, Borda score (the vertex-id order of
 *   Section 4), largest outgoing / incoming edge weight, the initialisation
 *   filter of Section 4 (1 if the largest incoming weight exceeds the largest
 *   outgoing one: x cannot win), mean outgoing / incoming weight, smallest /
 *   largest margin, log(m)/10, Copeland / max, Borda / max, largest outgoing
 *   weight / max, (largest outgoing - largest incoming) / n, 1.
 * Counts are scaled by 1/n_voters and by 1/(m-1) where they sum over
 * candidates.  feat: m x 16 floats, row-major, device memory.
 */
int schulze_features(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                     int dtype, int mode, float n_voters, float *feat);

/*
 * Learned proposer: a 16 -> 128 -> 128 -> 1 ReLU network, BF16 MFMA products
 * with FP32 accumulation, FP32 master parameters in one array of
 * schulze_mlp_param_count() floats laid out as
 *   W1[16][128] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3[1].
 * Inputs and the hidden activations are rounded to BF16 (nearest even), as
 * are W1, W2, W3 and the backward activations dz2, dz1.
 */
int schulze_mlp_param_count(void);

/* score[r] = network output for feature row r (feat: M x 16 floats). */
int schulze_mlp_forward(schulze_ctx *ctx, void *stream, const float *params, const float *feat,
                        int64_t M, float *score);

/* Segmented softmax cross-entropy over E elections, rows off[e] .. off[e+1]-1
 * (off: E+1 device int64), winner[r] = 1 for the election's Schulze winners:
 * loss[e] = log sum_rows exp(score) - log sum_winners exp(score);
 * dscore = gradient of the mean loss.  Elections without a marked winner get
 * loss 0 and zero gradient. */
int schulze_mlp_loss(schulze_ctx *ctx, void *stream, const float *score, const int64_t *offsets,
                     const uint8_t *winner, int32_t E, float *dscore, float *loss);

/* grad = gradient of sum_r dscore[r] * score[r] with respect to params
 * (deterministic: fixed per-workgroup partials reduced in a fixed order). */
int schulze_mlp_backward(schulze_ctx *ctx, void *stream, const float *params, const float *feat,
                         int64_t M, const float *dscore, float *grad);

/* One Adam step (bias-corrected, step >= 1) on the FP32 parameters. */
int schulze_mlp_adam(schulze_ctx *ctx, void *stream, float *params, const float *grad,
                     float *adam_m, float *adam_v, float lr, float beta1, float beta2, float eps,
                     int32_t step);

/* The network and its optimizer state for schulze_mlp_train_step.  Every
 * pointer is device memory the caller owns; params, adam_m, adam_v and grad
 * hold schulze_mlp_param_count() floats each. */
typedef struct {
    float *params;        /* FP32 master parameters (updated in place) */
    float *adam_m;        /* Adam first moments (zero before the first step) */
    float *adam_v;        /* Adam second moments (zero before the first step) */
    float *grad;          /* output: the step's gradient of the mean loss */
    int32_t *step;        /* one int32: Adam steps taken so far; each train step adds 1 and
                             uses the new value for the bias correction */
    float lr, beta1, beta2, eps;  /* lr > 0, 0 <= beta < 1, eps > 0 */
} schulze_mlp;

/* A minibatch of whole elections for schulze_mlp_train_step (device memory). */
typedef struct {
    const float *feat;      /* M x 16 feature rows (schulze_features), elections back to back */
    const int64_t *offsets; /* E + 1 row offsets: election e is rows offsets[e] .. offsets[e+1]-1,
                               offsets[0] = 0, offsets[E] = M */
    const uint8_t *winner;  /* M bytes: 1 for the election's Schulze winners */
    int64_t M;              /* rows, >= 1 */
    int32_t E;              /* elections, >= 1 */
} schulze_train_batch;

/*
 * One training step of the proposer: forward, the segmented loss of
 * schulze_mlp_loss (loss: E device floats, per election), backward to
 * net->grad, then Adam with the step counter advanced on the device.  The
 * same kernels as the separate calls, in the same order, so the result is
 * bitwise that of forward -> loss -> backward -> adam.  Nothing waits on the
 * host and the step count lives on the device, so a step can be captured in
 * a HIP graph once and replayed on new minibatches copied into the same
 * buffers (an earlier call with at least the same M must have sized the
 * workspace: 8 M bytes for scores and their gradient, plus the backward's
 * partials).
 */
int schulze_mlp_train_step(schulze_ctx *ctx, void *stream, const schulze_mlp *net,
                           const schulze_train_batch *b, float *loss);

/* Statistics of one schulze_winners_learned call. */
typedef struct {
    int32_t proposal;      /* first candidate the network proposed */
    int32_t first_hit;     /* 1 if that candidate is a winner */
    int32_t verify_calls;  /* exact checks run (proposal, climbs, tied candidates) */
    int32_t climbs;        /* moves to a beater */
    int32_t fallback;      /* 1 if the full closure decided */
    int32_t n_winners;
} schulze_learned_stats;

/*
 * Exact Schulze winners via a learned proposal.  The network (params, see
 * schulze_mlp_param_count) scores the features of d; the best candidate the
 * initialisation filter of Section 4 keeps is checked exactly
 * (schulze_verify_counts, then schulze_verify over written weights, see
 * below; schulze_set_proposer replaces the network by a plain score).
 * If it is beaten, the check moves to the highest-scored beater (at most
 * max_climb times); once a winner is found the candidates tied with it are
 * checked too (every winner is tied with every other winner).  If no winner
 * is found or more than max_tied candidates are tied, schulze_closure and
 * schulze_winners decide.  The result equals schulze_winners on the closure
 * for any network.  The search runs on the host and synchronises the
 * stream after each check; the winner set itself (is_winner, n_winners) is
 * written by work queued on the stream when the call returns (at most 64
 * winners; a larger set is copied before the call returns).
 * Returns SCHULZE_EDEVICE, with no winner set written, when the device error
 * word is set after a check (a widest-path launch gave up on its bounded
 * wait, or an earlier call left an error unread).
 *
 * n_voters   feature scale (number of voters).
 * is_winner  m device bytes.   n_winners: NULL or one device int32.
 * stats      NULL or host struct.
 * The first check is schulze_verify_counts (it reads d, nothing written);
 * later checks of the same call (climbs, tied candidates) write the weights
 * once and sweep over their rows.
 * Workspace: O(m); once a second check runs, int32 counts add m^2 int32
 * signed weights S = w - w^T (both weight rules give a pair an edge in at
 * most one direction, so w = max(S, 0) and w^T = max(-S, 0)) and 16-bit
 * counts 2 m^2 elements (w and w^T); m^2 elements more if the fallback runs.
 */
int schulze_winners_learned(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                            int dtype, int mode, float n_voters, const float *params,
                            int32_t max_climb, int32_t max_tied, uint8_t *is_winner,
                            int32_t *n_winners, schulze_learned_stats *stats);

/*
 * Proposer of schulze_winners_learned (the verification that follows is the
 * same for every proposer, so the winner set is too):
 *   NETWORK       the trained network's scores, best candidate the Section 4
 *                 initialisation filter keeps (default);
 *   BORDA         the Borda score, the vertex order Section 4 suggests;
 *   COPELAND      the Copeland score (pairwise wins);
 *   FILTER_BORDA  the filter of Section 4, then Borda.
 * The proposer's scores also pick the beater a failed check moves to (ties:
 * lowest id).  With a proposer other than NETWORK, params may be NULL.
 * Returns SCHULZE_EINVAL for other values.
 */
enum {
    SCHULZE_PROPOSER_NETWORK = 0,
    SCHULZE_PROPOSER_BORDA = 1,
    SCHULZE_PROPOSER_COPELAND = 2,
    SCHULZE_PROPOSER_FILTER_BORDA = 3
};
int schulze_set_proposer(schulze_ctx *ctx, int proposer);

/* Statistics of one schulze_winners_propagate call. */
typedef struct {
    int32_t rounds;     /* rounds of preprocessing, propagation and postprocessing */
    int32_t sweeps;     /* propagation sweeps over all rounds, both directions */
    int32_t n_winners;
} schulze_propagate_stats;

/*
 * Schulze winners by the paper's own winners-only algorithm (Section 4):
 * the initialisation filter, then rounds of forward/backward propagation of
 * the smallest label reaching (reached by) each vertex together with the
 * widest-path width from (to) that label's candidate, and postprocessing of
 * the labels, until no candidate is undecided.  Labels follow Borda scores
 * descending (ties by id) when borda_order != 0, else candidate ids.  Each
 * propagation runs to its fixpoint in one cooperative launch of dense
 * (max, min) sweeps over the weight matrix.  The result equals
 * schulze_winners on the closure.  Synchronises the stream (the rounds are
 * driven from the host).
 *
 * d, ldd, m, dtype, mode  as for schulze_closure (m <= 65534).
 * is_winner  m device bytes.   n_winners: NULL or one device int32.
 * stats      NULL or host struct.
 * Workspace: 2 m^2 elements of dtype plus O(m).
 */
int schulze_winners_propagate(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                              int dtype, int mode, int borda_order, uint8_t *is_winner,
                              int32_t *n_winners, schulze_propagate_stats *stats);

/* Statistics of one schulze_topk_propagate call. */
typedef struct {
    int32_t levels;  /* rounds of winner removal run */
    int32_t ranked;  /* candidates with a level (>= k unless fewer than k exist) */
    int32_t rounds;  /* propagation rounds over all levels */
    int32_t sweeps;  /* propagation sweeps over all levels, both directions */
} schulze_topk_stats;

/*
 * Top-k by iterated winner removal (the closing remark of Section 4):
 * level 0 is the set of Schulze winners; the winners are then taken out of
 * the election (their edges deleted) and level 1 is the set of Schulze
 * winners of the candidates left, and so on, until at least k candidates
 * have a level or none is left.  Each level runs the algorithm of
 * schulze_winners_propagate on the candidates still in.  Widest paths of a
 * later level avoid the removed candidates, so this order can differ from
 * the ranking of schulze_ranking (which orders by the full graph's widths).
 * Synchronises the stream.
 *
 * d, ldd, m, dtype, mode, borda_order  as for schulze_winners_propagate.
 * k       >= 1 (k >= m ranks everyone).
 * level   m device int32: the level of each candidate, -1 if not reached.
 * stats   NULL or host struct.
 * Errors: EINVAL for k < 1 or bad arguments; EUNSUPPORTED for m > 65534.
 * Workspace: as schulze_winners_propagate.
 */
int schulze_topk_propagate(schulze_ctx *ctx, void *stream, const void *d, int64_t ldd, int32_t m,
                           int dtype, int mode, int borda_order, int32_t k, int32_t *level,
                           schulze_topk_stats *stats);

/*
 * Closure schedule.  AUTO (default): one persistent cooperative launch whose
 * workgroups exchange the diagonal and panel tiles of each round through
 * device memory and flags, falling back to PHASED when the device refuses a
 * cooperative launch.  PHASED: three launches per round (diagonal, panels,
 * rest).  Both give identical results.
 */
enum { SCHULZE_SCHEDULE_AUTO = 0, SCHULZE_SCHEDULE_PHASED = 1 };
int schulze_set_closure_schedule(schulze_ctx *ctx, int schedule);

/*
 * Tile size B of the blocked closure (Section 5.2's recurrence cut into
 * B x B tiles): 0 (default) picks by value width and m (uint16: 128 from
 * m = 6144 on, else 64; int32: 128 from m = 2048 on, else 64), 64 or 128
 * force it.
 * Every B gives the same p; a larger B does more work per tile and round
 * and has fewer rounds, a smaller one more parallelism per round.  Returns
 * SCHULZE_EINVAL for other values.
 */
int schulze_set_closure_tile(schulze_ctx *ctx, int tile);

/*
 * Counting of truncated ballots over many candidates (the sparse form
 * d[x][y] = R_x - C[y][x] of Section 2.1's counts, chosen on the device when
 * the listed candidates of truncated ballots are too many for a dense count):
 * BUCKETED (default for m <= 32768 and n * L <= 2^27) sorts the listed
 * entries by candidate and accumulates each candidate's row of C in LDS;
 * ATOMIC adds every pair with a device-wide atomic.  Both give the same d.
 */
enum { SCHULZE_SPARSE_BUCKETED = 0, SCHULZE_SPARSE_ATOMIC = 1 };
int schulze_set_sparse_count(schulze_ctx *ctx, int mode);

/*
 * Value ranking of int32 closures (default on).  The (max, min) recurrence
 * of Section 2.1 commutes with every strictly increasing map of the weights
 * that keeps 0, so when the weights of an int32 closure with m >= 1024 take
 * at most 65535 distinct nonzero values, all below 2^24, the closure runs on
 * the ranks of the values in packed uint16 and maps the result back: same
 * output, about a third less arithmetic per update.  The decision is taken
 * on the device (a 2 MB bitmap of the values and a count): both variants are
 * queued and the one not needed returns at once, so the call stays
 * asynchronous and can be captured in a HIP graph.  With ranking off, or
 * when the values do not fit, the int32 closure runs.
 * Workspace when ranking: 2 m_p^2 + 4.2 MB bytes on top of the closure's
 * (m_p = m rounded up to the tile size), reserved before any work is queued.
 */
int schulze_set_value_ranking(schulze_ctx *ctx, int enable);

/*
 * Value width the last schulze_closure call on this context ran the
 * recurrence in: 16 (uint16 counts, or int32 weights replaced by their
 * ranks), 32 (int32), or 0 if no closure has run.  Synchronises `stream`
 * when the decision was taken on the device.
 */
int schulze_closure_value_bits(schulze_ctx *ctx, void *stream, int32_t *value_bits);

/*
 * Limits of the frontier sweeps' bounded waits, for tests of their failure
 * paths (callers that test how a stuck or runaway sweep is reported; not
 * for normal use).  The sweeps of schulze_widest_from, schulze_verify,
 * schulze_verify_noalloc, schulze_winners_learned, schulze_winners_propagate
 * and schulze_topk_propagate meet at a grid barrier once per sweep; a
 * workgroup that polls the barrier more than spin_limit times, or a run
 * that reaches max_sweeps sweeps with a frontier left (impossible for a
 * correct run: widths only grow), stops every workgroup of the launch,
 * leaves its outputs unwritten and sets SCHULZE_EDEVICE in the device error
 * word; the learned and propagation calls then return SCHULZE_EDEVICE
 * instead of deciding on the partial result.  0 restores a default (2^24
 * polls; m + 1 or 2 m + 2 sweeps).  Negative values: SCHULZE_EINVAL.
 */
int schulze_set_sweep_limits(schulze_ctx *ctx, int64_t spin_limit, int32_t max_sweeps);

/*
 * Batches of independent elections (Section 2.1 applied to each election of
 * the batch), run by one persistent launch whose workgroups take work items
 * from a queue: ballot scans, pairwise counts split into runs of candidate
 * sub-blocks and voter ranges, and per election one workgroup for weights,
 * closure, winners and ranking.  Results equal schulze_pairwise,
 * schulze_closure, schulze_winners and schulze_ranking applied election by
 * election (int32 counts).
 */
#define SCHULZE_BATCH_MAX_M 1024

/* One election of a batch.  Offsets are in elements of the arrays they index. */
typedef struct {
    int64_t ballot_off; /* first entry of the election's n x L ballots in `ballots` */
    int64_t n;          /* ballots (voters), 0 <= n < 2^31 */
    int32_t L;          /* entries per ballot, 1 <= L <= m */
    int32_t m;          /* candidates, 1 <= m <= SCHULZE_BATCH_MAX_M */
    int64_t mat_off;    /* first element of the election's m x m blocks (row pitch m) in d and p */
    int64_t vec_off;    /* first element of its m-entry blocks in is_winner, beaten_by, order, level */
} schulze_election;

typedef struct {
    int32_t max_range_pairs; /* 0 = automatic; else at most this many voter pairs per counting range */
    int32_t closure_only;    /* 1 = the plan only serves runs without ballots (no rank-pair buffer) */
    int32_t topk;            /* 0 = no levels; k > 0: runs given a level array rank at least k candidates
                                per election by iterated winner removal (as schulze_topk_propagate) */
    int32_t reserved[5];     /* zero */
} schulze_batch_options;

typedef struct schulze_batch schulze_batch;

/*
 * Plan a batch: validate the descriptors (host memory, E entries), choose per
 * election the counting layout and the closure schedule (see
 * schulze_batch_set_closure), order the work largest election first, and
 * allocate the plan's device memory: about n*m*2 bytes of rank pairs per
 * election, one closure matrix per resident workgroup, counters.
 *
 * Ballots follow schulze_pairwise (ids best first, padding ends a ballot), with
 * two batch rules: an id after a padding entry is an invalid ballot, and an
 * election with L >= m-1 is taken as complete rankings, so each of its
 * ballots must list at least m-1 candidates (the unlisted one is last);
 * elections with L < m-1 may end ballots early.  Voter weights are not
 * supported.  Counts of elections with n <= 65535 run the closure on uint16,
 * others on int32.
 * ballot_dtype  SCHULZE_U16 or SCHULZE_I32; mode  schulze_weight_mode.
 * opt           NULL for defaults.
 */
int schulze_batch_plan(schulze_ctx *ctx, const schulze_election *elections, int32_t E,
                       int ballot_dtype, int mode, const schulze_batch_options *opt,
                       schulze_batch **plan);

/* Free a plan (synchronises the device).  NULL is accepted. */
void schulze_batch_destroy(schulze_batch *plan);

enum { SCHULZE_BATCH_GRAPH = 1 };

/*
 * Run a planned batch on `stream`.
 *
 * ballots    device ballots addressed by the descriptors, or NULL: then d is
 *            an INPUT (counts of each election, e.g. from an earlier run; each
 *            count at most the election's n) and only weights, closure,
 *            winners and ranking run.
 * d          int32 counts, written when ballots != NULL (d[x][x] = 0).
 * p          NULL or int32 closures (p[x][x] = 0).
 * is_winner  1 for Schulze winners, else 0.     n_winners: NULL or E int32.
 * beaten_by  NULL or int32 (candidates beating x).  order: NULL or int32
 *            (candidates by beaten_by, then id), as schulze_ranking.
 * level      NULL or int32 top-k levels (plans made with topk > 0 only, else
 *            SCHULZE_EINVAL): level 0 = the winners; then, with the ranked
 *            candidates and their edges taken out, the winners of the rest
 *            (closing remark of Section 4), until at least topk candidates of
 *            the election are ranked; -1 for candidates not reached.  Each
 *            level closes the election's weights once more.
 * All are device pointers that the descriptors' offsets index; the caller
 * sizes them.  Invalid ballots set the device error word to SCHULZE_EBALLOT.
 * flags      SCHULZE_BATCH_GRAPH: capture the reset of the plan's counters and
 *            the persistent launch in a HIP graph on first use (again when any
 *            pointer argument changes) and launch the graph; 0: launch directly.
 * Calls on one plan must not overlap (the plan owns the queue counters).
 */
int schulze_batch_run(schulze_ctx *ctx, void *stream, schulze_batch *plan, const void *ballots,
                      int32_t *d, int32_t *p, uint8_t *is_winner, int32_t *n_winners,
                      int32_t *beaten_by, int32_t *order, int32_t *level, int flags);

/*
 * Closure schedules of a batch election, chosen per value width (16 or 32
 * bits) and per bucket of 32 candidate counts (1-32, 33-64, ...):
 *   REGISTERS  plain Floyd-Warshall recurrence with the matrix, padded to a
 *              multiple of 32, in the registers of one workgroup (at most
 *              192 candidates for 16-bit values, 128 for 32-bit);
 *   TILED32/64/128  three-phase blocked recurrence with tiles of that size
 *              (TILED32 and TILED128 for 16-bit values only).
 * AUTO (-1) restores the built-in choice.  Plans read the table when created.
 */
enum {
    SCHULZE_BATCH_CLOSURE_AUTO = -1,
    SCHULZE_BATCH_CLOSURE_REGISTERS = 0,
    SCHULZE_BATCH_CLOSURE_TILED32 = 1,
    SCHULZE_BATCH_CLOSURE_TILED64 = 2,
    SCHULZE_BATCH_CLOSURE_TILED128 = 3
};
int schulze_batch_set_closure(schulze_ctx *ctx, int32_t value_bits, int32_t m_lo, int32_t m_hi,
                              int32_t variant);
/* The schedule a plan would use for an election of m candidates. */
int schulze_batch_get_closure(schulze_ctx *ctx, int32_t value_bits, int32_t m, int32_t *variant);

/*
 * Autotuner: for each bucket of 32 candidate counts up to m_max, time every
 * schedule that applies on a closure-only batch of one election per resident
 * workgroup (pseudo-random tournament counts at the bucket's largest m) and
 * store the fastest in the context's table.  ms: NULL or host floats
 * [ceil(m_max/32)][4], the best of two timed runs per schedule in
 * milliseconds (-1 where a schedule does not apply).  Synchronises `stream`.
 */
int schulze_batch_autotune(schulze_ctx *ctx, void *stream, int32_t value_bits, int32_t m_max,
                           float *ms);

/*
 * Per-kernel timing (a profiling aid, off by default).  While enabled, every
 * kernel the library launches is bracketed by HIP events on its own stream;
 * schulze_kernel_time synchronises and returns the number of launches and
 * their summed duration (milliseconds) for the named kernel since the last
 * reset.  Names: "ballot_scan", "route", "ballot_scatter", "count_dense",
 * "count_trunc", "count_sparse", "count_finish", "weights", "fw_diag", "fw_panel",
 * "fw_rest", "fw_persist", "fw_store", "beaten_by", "rank_sort",
 * "winners", "fill", "widest", "verdict", "features", "mlp_prepare",
 * "mlp_forward", "mlp_backward", "mlp_loss", "mlp_adam", "propose", "batch"
 * (a batch run: the persistent launch, or the whole graph when captured),
 * "label_post" (schulze_winners_propagate's filter, order and
 * postprocessing kernels), "label_sweep" (its propagation launches),
 * "value_rank" (the value-ranking kernels of int32 closures),
 * "feature_rows" (the row pass of the per-candidate features),
 * "valu_probe".
 */
int schulze_set_timing(schulze_ctx *ctx, int enable);
int schulze_kernel_time(schulze_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms);
int schulze_reset_timing(schulze_ctx *ctx);

/*
 * Integer VALU throughput probe (a measurement aid for the rooflines of the
 * count and closure kernels, which are bound by the vector ALU): one launch
 * of `workgroups` workgroups of 256 threads, each lane running `trips` x 160
 * packed-uint16 max, min, add and subtract instructions on eight
 * independent chains.  *lane_ops (host) receives the number of lane
 * operations launched (workgroups x 256 x trips x 160); time the launch on
 * `stream` with events.  out: one device uint32 that the kernel may write
 * (it keeps the chains' results live).  EINVAL for null pointers or
 * non-positive sizes.
 */
int schulze_valu_probe(schulze_ctx *ctx, void *stream, int32_t workgroups, int64_t trips, uint32_t *out,
                       int64_t *lane_ops);

#ifdef __cplusplus
}
#endif

#endif /* SCHULZE_H */
