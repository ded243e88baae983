// Learned winner proposer: a 16 -> 128 -> 128 -> 1 ReLU network over the
// per-candidate features, with hand-written BF16 MFMA GEMMs (FP32
// accumulation) for the forward pass, the backward pass and a segmented
// softmax loss over elections, plus Adam with FP32 master weights.
//
// Parameter layout (FP32, SCHULZE_MLP_PARAMS floats):
//   W1[16][128] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3[1]
// z1 = x W1 + b1, h1 = relu(z1), z2 = h1 W2 + b2, h2 = relu(z2), s = h2 W3 + b3.
// Rounding points (the CPU reference applies the same ones): x, W1, W2, W3,
// h1, h2, dz2 and dz1 are rounded to BF16 (nearest even); products are
// accumulated in FP32; biases stay FP32.
//
// MFMA lane layouts on gfx950 (checked on the device):
//   v_mfma_f32_32x32x16_bf16: lane l supplies A row l%32 / B column l%32 with
//   k = 8 (l/32) + e, e < 8; D element i of lane l is row 8 (i/4) + 4 (l/32)
//   + i%4, column l%32.
//   v_mfma_f32_16x16x32_bf16: lane l supplies row/column l%16 with
//   k = 8 (l/16) + e; D element i of lane l is row 4 (l/16) + i, column l%16.
#include "internal.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NF = 16, NH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NF * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
constexpr int ROWS = 64;            // rows per tile
constexpr int PH = NH + 8;          // padded LDS pitch (bf16) of 128-wide rows
constexpr int PF = NF + 8;          // padded pitch of 16-wide rows
constexpr int PR = ROWS + 8;        // padded pitch of 64-wide (row index) rows

__device__ inline bf16 to_bf16(float f) { return (bf16)f; }
__device__ inline float from_bf16(bf16 b) { return (float)b; }

__device__ inline bf16x8 ld8(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// BF16 copies of the weights in the layouts the kernels read:
// w1t[j][f] = W1[f][j], w2t[j][i] = W2[i][j], w2[i][j] = W2[i][j], w3[j].
struct NetBf16 {
    bf16 *w1t, *w2t, *w2, *w3;
};

__global__ __launch_bounds__(256) void k_mlp_prepare(const float *__restrict__ p, NetBf16 q) {
    for (int t = blockIdx.x * 256 + threadIdx.x; t < NH * NH; t += gridDim.x * 256) {
        const int i = t / NH, j = t % NH;
        const bf16 v = to_bf16(p[OFF_W2 + i * NH + j]);
        q.w2[i * NH + j] = v;
        q.w2t[j * NH + i] = v;
        if (i < NF) q.w1t[j * NF + i] = to_bf16(p[OFF_W1 + i * NH + j]);
        if (i == 0) q.w3[j] = to_bf16(p[OFF_W3 + j]);
    }
}

// Shared forward part of one 64-row tile.  On return: xs (bf16 inputs),
// h1 (bf16, row-major), z1 signs in m1, and per lane the layer-2 outputs
// h2 (bf16-rounded, as float) of its two 32 x 32 blocks plus their masks.
struct Lds {
    bf16 w1t[NH * PF];
    bf16 w2t[NH * PH];
    bf16 xs[ROWS * PF];
    bf16 h1[ROWS * PH];
    float part[ROWS][4];
};

__device__ inline void load_weights(Lds &L, const NetBf16 &q) {
    for (int t = threadIdx.x; t < NH * NH; t += 256) L.w2t[(t / NH) * PH + t % NH] = q.w2t[t];
    for (int t = threadIdx.x; t < NH * NF; t += 256) L.w1t[(t / NF) * PF + t % NF] = q.w1t[t];
}

__device__ inline void load_tile(Lds &L, const float *__restrict__ X, int64_t row0, int64_t M) {
    for (int t = threadIdx.x; t < ROWS * NF; t += 256) {
        const int r = t / NF, f = t % NF;
        const int64_t row = row0 + r;
        L.xs[r * PF + f] = to_bf16(row < M ? X[row * NF + f] : 0.0f);
    }
}

// Wave w: row block rb = w >> 1, column blocks 2 (w & 1) + {0, 1}.
__device__ inline void forward_tile(Lds &L, const float *__restrict__ b1, const float *__restrict__ b2,
                                    f32x16 (&h2)[2], uint32_t (&mask2)[2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rb = wave >> 1, hi = lane >> 5, lo = lane & 31;
    // layer 1: h1 = relu(x W1 + b1)
    for (int c = 0; c < 2; ++c) {
        const int cb = 2 * (wave & 1) + c;
        f32x16 acc = {};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&L.xs[(rb * 32 + lo) * PF + 8 * hi]),
                                                     ld8(&L.w1t[(cb * 32 + lo) * PF + 8 * hi]), acc, 0, 0, 0);
        const int col = cb * 32 + lo;
        const float bias = b1[col];
        for (int i = 0; i < 16; ++i) {
            const int row = rb * 32 + 8 * (i >> 2) + 4 * hi + (i & 3);
            L.h1[row * PH + col] = to_bf16(fmaxf(acc[i] + bias, 0.0f));
        }
    }
    __syncthreads();
    // layer 2: h2 = relu(h1 W2 + b2)
    for (int c = 0; c < 2; ++c) {
        const int cb = 2 * (wave & 1) + c;
        f32x16 acc = {};
        for (int kk = 0; kk < NH / 16; ++kk)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&L.h1[(rb * 32 + lo) * PH + 16 * kk + 8 * hi]),
                                                         ld8(&L.w2t[(cb * 32 + lo) * PH + 16 * kk + 8 * hi]), acc,
                                                         0, 0, 0);
        const float bias = b2[cb * 32 + lo];
        uint32_t mk = 0;
        for (int i = 0; i < 16; ++i) {
            const float z = acc[i] + bias;
            mk |= (z > 0.0f ? 1u : 0u) << i;
            h2[c][i] = from_bf16(to_bf16(fmaxf(z, 0.0f)));
        }
        mask2[c] = mk;
    }
}

// Sum over the 32 lanes of a half-wave (fixed butterfly order).
__device__ inline float half_sum(float v) {
    for (int off = 1; off < 32; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------------------ forward
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ p, NetBf16 q, const float *__restrict__ X,
                                                 int64_t M, float *__restrict__ score) {
    __shared__ Lds L;
    load_weights(L, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rb = wave >> 1, hi = lane >> 5, lo = lane & 31;
    const int64_t ntiles = (M + ROWS - 1) / ROWS;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();
        load_tile(L, X, t * ROWS, M);
        __syncthreads();
        f32x16 h2[2];
        uint32_t mk[2];
        forward_tile(L, p + OFF_B1, p + OFF_B2, h2, mk);
        // layer 3: s = h2 W3 + b3 (deterministic: lanes, then blocks in order)
        for (int c = 0; c < 2; ++c) {
            const int cb = 2 * (wave & 1) + c;
            const float w3 = from_bf16(q.w3[cb * 32 + lo]);
            for (int i = 0; i < 16; ++i) {
                const float sum = half_sum(h2[c][i] * w3);
                if (lo == 0) L.part[rb * 32 + 8 * (i >> 2) + 4 * hi + (i & 3)][cb] = sum;
            }
        }
        __syncthreads();
        if (threadIdx.x < ROWS) {
            const int64_t row = t * ROWS + threadIdx.x;
            const float *pp = L.part[threadIdx.x];
            if (row < M) score[row] = p[OFF_B3] + ((pp[0] + pp[1]) + (pp[2] + pp[3]));
        }
    }
}

// ------------------------------------------------------------------ loss
// One wavefront per election e over rows [off[e], off[e+1]): softmax
// cross-entropy with the probability mass of the winner set,
//   loss_e = log sum_all exp(s) - log sum_winners exp(s),
// ds = (softmax over all - softmax over winners, on winners) / E.
__global__ __launch_bounds__(256) void k_seg_loss(const float *__restrict__ score, const int64_t *__restrict__ off,
                                                  const uint8_t *__restrict__ winner, int32_t E,
                                                  float *__restrict__ ds, float *__restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int32_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= E) return;
    const int64_t a = off[e], b = off[e + 1];
    float mx = -INFINITY;
    for (int64_t r = a + lane; r < b; r += 64) mx = fmaxf(mx, score[r]);
    for (int o = 1; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float sa = 0.f, sw = 0.f;
    for (int64_t r = a + lane; r < b; r += 64) {
        const float ex = expf(score[r] - mx);
        sa += ex;
        if (winner[r]) sw += ex;
    }
    for (int o = 1; o < 64; o <<= 1) {
        sa += __shfl_xor(sa, o);
        sw += __shfl_xor(sw, o);
    }
    const float inv_e = 1.0f / (float)E;
    const bool ok = sw > 0.f;
    for (int64_t r = a + lane; r < b; r += 64) {
        const float ex = expf(score[r] - mx);
        float g = ex / sa;
        if (winner[r] && ok) g -= ex / sw;
        ds[r] = ok ? g * inv_e : 0.f;
    }
    if (lane == 0) loss[e] = ok ? logf(sa) - logf(sw) : 0.f;
}

// ------------------------------------------------------------------ backward
// Persistent workgroups; each walks a fixed set of tiles (deterministic),
// recomputes the forward part, and accumulates its parameter-gradient
// partials in registers, written once at the end to partial[block][NPARAM].
struct BwdLds {
    Lds f;
    bf16 dz2[ROWS * PH];   // row-major
    bf16 dz2t[NH * PR];    // transposed
    bf16 h1t[NH * PR];     // transposed h1
    bf16 dz1t[NH * PR];    // transposed dz1
    bf16 xt[NF * PR];      // transposed inputs
    float ds[ROWS];
    float red[4][NH];
};

__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ p, NetBf16 q, const float *__restrict__ X,
                                                 const float *__restrict__ dsg, int64_t M,
                                                 float *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    BwdLds &L = *reinterpret_cast<BwdLds *>(smem);
    load_weights(L.f, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rb = wave >> 1, hi = lane >> 5, lo = lane & 31;
    // B operands of dh1 = dz2 W2^T stay in registers: W2[i][16 kk + 8 hi ..]
    bf16x8 w2f[2][NH / 16];
    for (int c = 0; c < 2; ++c)
        for (int kk = 0; kk < NH / 16; ++kk)
            w2f[c][kk] = ld8(&q.w2[(int64_t)((2 * (wave & 1) + c) * 32 + lo) * NH + 16 * kk + 8 * hi]);

    f32x16 gw2[4] = {};     // dW2 blocks (ib = wave, jb = 0..3)
    f32x4 gw1[2] = {};      // dW1 blocks (16 x 16): ib = 2 wave + {0,1}
    float gw3[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f}, gb1[2] = {0.f, 0.f}, gb3 = 0.f;

    const int64_t ntiles = (M + ROWS - 1) / ROWS;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();
        load_tile(L.f, X, t * ROWS, M);
        if (threadIdx.x < ROWS) {
            const int64_t row = t * ROWS + threadIdx.x;
            L.ds[threadIdx.x] = row < M ? dsg[row] : 0.f;
        }
        __syncthreads();
        f32x16 h2[2];
        uint32_t mk2[2];
        forward_tile(L.f, p + OFF_B1, p + OFF_B2, h2, mk2);
        // dz2 = mask2 * ds * w3; dW3 += h2 ds; db2 += dz2 (from the rounded dz2)
        for (int c = 0; c < 2; ++c) {
            const int cb = 2 * (wave & 1) + c;
            const int col = cb * 32 + lo;
            const float w3 = from_bf16(q.w3[col]);
            float s3 = 0.f, s2 = 0.f;
            for (int i = 0; i < 16; ++i) {
                const int row = rb * 32 + 8 * (i >> 2) + 4 * hi + (i & 3);
                const float dsr = L.ds[row];
                s3 += h2[c][i] * dsr;
                const bf16 dz = to_bf16(((mk2[c] >> i) & 1u) ? dsr * w3 : 0.0f);
                s2 += from_bf16(dz);
                L.dz2[row * PH + col] = dz;
                L.dz2t[col * PR + row] = dz;
            }
            gw3[c] += s3;
            gb2[c] += s2;
        }
        // transposed h1 and x for the weight-gradient products
        for (int e = threadIdx.x; e < ROWS * NH; e += 256) {
            const int r = e / NH, i = e % NH;
            L.h1t[i * PR + r] = L.f.h1[r * PH + i];
        }
        for (int e = threadIdx.x; e < ROWS * NF; e += 256) {
            const int r = e / NF, f = e % NF;
            L.xt[f * PR + r] = L.f.xs[r * PF + f];
        }
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int r = 0; r < ROWS; ++r) s += L.ds[r];
            gb3 += s;
        }
        __syncthreads();
        // dW2[i][j] += sum_rows h1[r][i] dz2[r][j]; wave owns i-block = wave
        for (int jb = 0; jb < 4; ++jb)
            for (int kk = 0; kk < ROWS / 16; ++kk)
                gw2[jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    ld8(&L.h1t[(wave * 32 + lo) * PR + 16 * kk + 8 * hi]),
                    ld8(&L.dz2t[(jb * 32 + lo) * PR + 16 * kk + 8 * hi]), gw2[jb], 0, 0, 0);
        // dh1 = dz2 W2^T; dz1 = mask1 * dh1 (mask1 from h1 > 0)
        for (int c = 0; c < 2; ++c) {
            const int ib = 2 * (wave & 1) + c;
            f32x16 acc = {};
            for (int kk = 0; kk < NH / 16; ++kk)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&L.dz2[(rb * 32 + lo) * PH + 16 * kk + 8 * hi]),
                                                             w2f[c][kk], acc, 0, 0, 0);
            const int col = ib * 32 + lo;
            float s1 = 0.f;
            for (int i = 0; i < 16; ++i) {
                const int row = rb * 32 + 8 * (i >> 2) + 4 * hi + (i & 3);
                const bool on = from_bf16(L.f.h1[row * PH + col]) > 0.0f;
                const bf16 dz = to_bf16(on ? acc[i] : 0.0f);
                s1 += from_bf16(dz);
                L.dz1t[col * PR + row] = dz;
            }
            gb1[c] += s1;
        }
        __syncthreads();
        // dW1[f][i] += sum_rows x[r][f] dz1[r][i] (16 x 16 blocks, k = rows)
        for (int c = 0; c < 2; ++c) {
            const int ib = 2 * wave + c;
            for (int kk = 0; kk < ROWS / 32; ++kk)
                gw1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    ld8(&L.xt[(lane & 15) * PR + 32 * kk + 8 * (lane >> 4)]),
                    ld8(&L.dz1t[(ib * 16 + (lane & 15)) * PR + 32 * kk + 8 * (lane >> 4)]), gw1[c], 0, 0, 0);
        }
    }
    // write this workgroup's partials (fixed order reductions only)
    float *out = partial + (int64_t)blockIdx.x * NPARAM;
    for (int jb = 0; jb < 4; ++jb)
        for (int i = 0; i < 16; ++i) {
            const int r = wave * 32 + 8 * (i >> 2) + 4 * hi + (i & 3);
            out[OFF_W2 + r * NH + jb * 32 + lo] = gw2[jb][i];
        }
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 4; ++i) {
            const int f = 4 * (lane >> 4) + i;
            out[OFF_W1 + f * NH + (2 * wave + c) * 16 + (lane & 15)] = gw1[c][i];
        }
    // bias and W3 gradients: combine the two half-waves and the two row blocks
    __syncthreads();
    for (int c = 0; c < 2; ++c) {
        const int col = (2 * (wave & 1) + c) * 32 + lo;
        // slot: row block rb, half hi -> red[2 rb + hi][col]
        L.red[2 * rb + hi][col] = gw3[c];
    }
    __syncthreads();
    if (threadIdx.x < NH) {
        const int col = threadIdx.x;
        out[OFF_W3 + col] = (L.red[0][col] + L.red[1][col]) + (L.red[2][col] + L.red[3][col]);
    }
    __syncthreads();
    for (int c = 0; c < 2; ++c) L.red[2 * rb + hi][(2 * (wave & 1) + c) * 32 + lo] = gb2[c];
    __syncthreads();
    if (threadIdx.x < NH) {
        const int col = threadIdx.x;
        out[OFF_B2 + col] = (L.red[0][col] + L.red[1][col]) + (L.red[2][col] + L.red[3][col]);
    }
    __syncthreads();
    for (int c = 0; c < 2; ++c) L.red[2 * rb + hi][(2 * (wave & 1) + c) * 32 + lo] = gb1[c];
    __syncthreads();
    if (threadIdx.x < NH) {
        const int col = threadIdx.x;
        out[OFF_B1 + col] = (L.red[0][col] + L.red[1][col]) + (L.red[2][col] + L.red[3][col]);
    }
    if (threadIdx.x == 0) out[OFF_B3] = gb3;
}

// grad[k] = sum over blocks of partial[block][k], in block order.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, int32_t nblocks,
                                                    float *__restrict__ grad) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * NPARAM + k];
    grad[k] = s;
}

// Adam (FP32 master weights), bias-corrected, step t >= 1: t_host, or the
// device counter *t_dev when given (the train step advances it first).
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m1, float *__restrict__ m2, float lr, float b1,
                                              float b2, float eps, int32_t t_host, const int32_t *__restrict__ t_dev) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= NPARAM) return;
    const int32_t t = t_dev ? *t_dev : t_host;
    const float gk = g[k];
    const float a = b1 * m1[k] + (1.f - b1) * gk;
    const float v = b2 * m2[k] + (1.f - b2) * gk * gk;
    m1[k] = a;
    m2[k] = v;
    const float ah = a / (1.f - powf(b1, (float)t));
    const float vh = v / (1.f - powf(b2, (float)t));
    p[k] -= lr * ah / (sqrtf(vh) + eps);
}

// The train step's Adam counter: one more step.
__global__ void k_step_next(int32_t *__restrict__ step) {
    if (threadIdx.x == 0) step[0] += 1;
}

size_t bwd_lds_bytes() { return sizeof(BwdLds); }

int prepare(schulze_ctx *ctx, hipStream_t s, const float *params, NetBf16 &q) {
    const size_t w2b = sizeof(bf16) * NH * NH, w1b = sizeof(bf16) * NH * NF;
    int rc = ws_reserve(ctx, WS_MLP, 2 * w2b + w1b + 256 + 256);
    if (rc != SCHULZE_OK) return rc;
    char *b = static_cast<char *>(ctx->ws[WS_MLP]);
    q.w2t = reinterpret_cast<bf16 *>(b);
    q.w2 = reinterpret_cast<bf16 *>(b + w2b);
    q.w1t = reinterpret_cast<bf16 *>(b + 2 * w2b);
    q.w3 = reinterpret_cast<bf16 *>(b + 2 * w2b + w1b + 256);
    SCHULZE_LAUNCH(ctx, K_MLP_PREP, s, k_mlp_prepare<<<dim3(16), dim3(256), 0, s>>>(params, q));
    return SCHULZE_OK;
}

int grid_for(schulze_ctx *ctx, int64_t M) {
    int64_t g = std::min<int64_t>((M + ROWS - 1) / ROWS, (int64_t)ctx->num_cus * 2);
    return (int)std::max<int64_t>(g, 1);
}

}  // namespace

extern "C" int schulze_mlp_forward(schulze_ctx *ctx, void *stream, const float *params, const float *feat, int64_t M,
                                   float *score) {
    if (!ctx || !params || !feat || !score || M < 0) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    if (M == 0) return SCHULZE_OK;
    hipStream_t s = (hipStream_t)stream;
    NetBf16 q;
    int rc = prepare(ctx, s, params, q);
    if (rc != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_MLP_FWD, s,
                   k_mlp_fwd<<<dim3((unsigned)grid_for(ctx, M)), dim3(256), 0, s>>>(params, q, feat, M, score));
    return SCHULZE_OK;
}

namespace {

// Backward of the prepared network (q) into grad; arguments checked.
int backward(schulze_ctx *ctx, hipStream_t s, const float *params, const NetBf16 &q, const float *feat, int64_t M,
             const float *dscore, float *grad) {
    int rc;
    const int G = grid_for(ctx, M);
    if ((rc = ws_reserve(ctx, WS_MLP_PARTIAL, sizeof(float) * (size_t)G * NPARAM)) != SCHULZE_OK) return rc;
    float *partial = static_cast<float *>(ctx->ws[WS_MLP_PARTIAL]);
    const size_t lds = bwd_lds_bytes();
    if (hipFuncSetAttribute((const void *)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return SCHULZE_EDEVICE;
    SCHULZE_LAUNCH(ctx, K_MLP_BWD, s,
                   k_mlp_bwd<<<dim3((unsigned)G), dim3(256), lds, s>>>(params, q, feat, dscore, M, partial));
    SCHULZE_LAUNCH(ctx, K_MLP_BWD, s,
                   k_mlp_reduce<<<dim3((unsigned)ceil_div(NPARAM, 256)), dim3(256), 0, s>>>(partial, G, grad));
    return SCHULZE_OK;
}

}  // namespace

extern "C" int schulze_mlp_backward(schulze_ctx *ctx, void *stream, const float *params, const float *feat, int64_t M,
                                    const float *dscore, float *grad) {
    if (!ctx || !params || !feat || !dscore || !grad || M < 0) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    NetBf16 q;
    int rc = prepare(ctx, s, params, q);
    if (rc != SCHULZE_OK) return rc;
    return backward(ctx, s, params, q, feat, M, dscore, grad);
}

extern "C" int schulze_mlp_loss(schulze_ctx *ctx, void *stream, const float *score, const int64_t *offsets,
                                const uint8_t *winner, int32_t E, float *dscore, float *loss) {
    if (!ctx || !score || !offsets || !winner || !dscore || !loss || E < 1) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    SCHULZE_LAUNCH(ctx, K_MLP_LOSS, s,
                   k_seg_loss<<<dim3((unsigned)ceil_div(E, 4)), dim3(256), 0, s>>>(score, offsets, winner, E, dscore,
                                                                                    loss));
    return SCHULZE_OK;
}

extern "C" int schulze_mlp_adam(schulze_ctx *ctx, void *stream, float *params, const float *grad, float *adam_m,
                                float *adam_v, float lr, float beta1, float beta2, float eps, int32_t step) {
    if (!ctx || !params || !grad || !adam_m || !adam_v || step < 1) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    SCHULZE_LAUNCH(ctx, K_MLP_ADAM, s,
                   k_adam<<<dim3((unsigned)ceil_div(NPARAM, 256)), dim3(256), 0, s>>>(params, grad, adam_m, adam_v, lr,
                                                                                     beta1, beta2, eps, step,
                                                                                     nullptr));
    return SCHULZE_OK;
}

extern "C" int schulze_mlp_train_step(schulze_ctx *ctx, void *stream, const schulze_mlp *net,
                                      const schulze_train_batch *b, float *loss) {
    if (!ctx || !net || !b || !loss) return SCHULZE_EINVAL;
    if (!net->params || !net->adam_m || !net->adam_v || !net->grad || !net->step) return SCHULZE_EINVAL;
    if (!b->feat || !b->offsets || !b->winner || b->M < 1 || b->E < 1) return SCHULZE_EINVAL;
    if (!(net->lr > 0.f) || !(net->beta1 >= 0.f && net->beta1 < 1.f) || !(net->beta2 >= 0.f && net->beta2 < 1.f) ||
        !(net->eps > 0.f))
        return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    // scores and their gradient live in the workspace
    const size_t vec = round_up(sizeof(float) * (size_t)b->M, 256);
    int rc = ws_reserve(ctx, WS_MLP_TRAIN, 2 * vec);
    if (rc != SCHULZE_OK) return rc;
    float *score = static_cast<float *>(ctx->ws[WS_MLP_TRAIN]);
    float *dscore = reinterpret_cast<float *>(static_cast<char *>(ctx->ws[WS_MLP_TRAIN]) + vec);
    NetBf16 q;
    if ((rc = prepare(ctx, s, net->params, q)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_MLP_FWD, s,
                   k_mlp_fwd<<<dim3((unsigned)grid_for(ctx, b->M)), dim3(256), 0, s>>>(net->params, q, b->feat, b->M,
                                                                                       score));
    SCHULZE_LAUNCH(ctx, K_MLP_LOSS, s,
                   k_seg_loss<<<dim3((unsigned)ceil_div(b->E, 4)), dim3(256), 0, s>>>(score, b->offsets, b->winner,
                                                                                       b->E, dscore, loss));
    if ((rc = backward(ctx, s, net->params, q, b->feat, b->M, dscore, net->grad)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_MLP_ADAM, s, k_step_next<<<dim3(1), dim3(64), 0, s>>>(net->step));
    SCHULZE_LAUNCH(ctx, K_MLP_ADAM, s,
                   k_adam<<<dim3((unsigned)ceil_div(NPARAM, 256)), dim3(256), 0, s>>>(
                       net->params, net->grad, net->adam_m, net->adam_v, net->lr, net->beta1, net->beta2, net->eps, 0,
                       net->step));
    return SCHULZE_OK;
}

extern "C" int schulze_mlp_param_count(void) { return NPARAM; }
