// Context, workspace, device error word and kernel timing of the C ABI.
#include <string.h>

#include <new>

#include "internal.h"

const char *const kKernelNames[K_NUM_KERNELS] = {
    "ballot_scan", "ballot_scatter", "count_dense", "count_sparse", "count_finish", "weights",
    "fw_diag",     "fw_panel",       "fw_rest",     "fw_store",     "beaten_by",    "rank_sort",
    "winners",     "fill",           "fw_persist",  "route",        "count_trunc",
    "widest",      "verdict",        "features",    "mlp_prepare",  "mlp_forward",
    "mlp_backward", "mlp_loss",      "mlp_adam",    "propose",     "batch",
    "label_post",   "label_sweep", "value_rank", "feature_rows", "valu_probe"};

extern "C" const char *schulze_strerror(int code) {
    switch (code) {
        case SCHULZE_OK: return "ok";
        case SCHULZE_EINVAL: return "invalid argument";
        case SCHULZE_ERANGE: return "counts do not fit the requested dtype";
        case SCHULZE_ENOMEM: return "out of device memory";
        case SCHULZE_EDEVICE: return "HIP runtime error";
        case SCHULZE_EBALLOT: return "invalid ballot (id out of range or listed twice)";
        case SCHULZE_EUNSUPPORTED: return "unsupported request";
        default: return "unknown error";
    }
}

int bind_device(schulze_ctx *ctx) {
    return hipSetDevice(ctx->device) == hipSuccess ? SCHULZE_OK : SCHULZE_EDEVICE;
}

int launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SCHULZE_OK : SCHULZE_EDEVICE;
}

extern "C" int schulze_create(schulze_ctx **out, int device) {
    if (!out) return SCHULZE_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SCHULZE_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return SCHULZE_EDEVICE;
    schulze_ctx *ctx = new (std::nothrow) schulze_ctx();
    if (!ctx) return SCHULZE_ENOMEM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return SCHULZE_EDEVICE;
    }
    ctx->num_cus = prop.multiProcessorCount;
    if (hipMalloc((void **)&ctx->err, sizeof(int32_t)) != hipSuccess) {
        delete ctx;
        return SCHULZE_ENOMEM;
    }
    if (hipMemset(ctx->err, 0, sizeof(int32_t)) != hipSuccess) {
        (void)hipFree(ctx->err);
        delete ctx;
        return SCHULZE_EDEVICE;
    }
    ctx->launches.assign(K_NUM_KERNELS, 0);
    ctx->total_ms.assign(K_NUM_KERNELS, 0.0);
    if (verify_scratch_init(device, &ctx->verify_scratch) != SCHULZE_OK) {
        (void)hipFree(ctx->err);
        delete ctx;
        return SCHULZE_EDEVICE;
    }
    *out = ctx;
    return SCHULZE_OK;
}

extern "C" void schulze_destroy(schulze_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < WS_NUM_SLOTS; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    for (auto &p : ctx->pending) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    (void)hipFree(ctx->err);
    delete ctx;
}

int ws_reserve(schulze_ctx *ctx, WsSlot slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ctx->ws_bytes[slot] >= bytes) return SCHULZE_OK;
    if (ctx->ws[slot]) {
        // the old buffer may still be read by queued work
        if (hipDeviceSynchronize() != hipSuccess) return SCHULZE_EDEVICE;
        (void)hipFree(ctx->ws[slot]);
        ctx->ws[slot] = nullptr;
        ctx->ws_bytes[slot] = 0;
    }
    size_t want = (size_t)round_up((int64_t)bytes, 1 << 20);
    if (hipMalloc(&ctx->ws[slot], want) != hipSuccess) {
        (void)hipGetLastError();
        return SCHULZE_ENOMEM;
    }
    ctx->ws_bytes[slot] = want;
    return SCHULZE_OK;
}

extern "C" int schulze_get_device_error(schulze_ctx *ctx, void *stream, int32_t *err_host) {
    if (!ctx || !err_host) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    int32_t v = 0;
    if (hipMemcpyAsync(&v, ctx->err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return SCHULZE_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return SCHULZE_EDEVICE;
    if (v != 0) {
        int rc = fill_u32(ctx, s, (uint32_t *)ctx->err, 1, 0u);
        if (rc != SCHULZE_OK) return rc;
        if (hipStreamSynchronize(s) != hipSuccess) return SCHULZE_EDEVICE;
    }
    *err_host = v;
    return SCHULZE_OK;
}

// ---------------------------------------------------------------- fill

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t words, uint32_t value) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    uint4 v4 = make_uint4(value, value, value, value);
    size_t n4 = words / 4;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);
    if (((uintptr_t)p & 15) == 0) {
        for (size_t j = i; j < n4; j += stride) p4[j] = v4;
        for (size_t j = n4 * 4 + i; j < words; j += stride) p[j] = value;
    } else {
        for (size_t j = i; j < words; j += stride) p[j] = value;
    }
}

int fill_u32(schulze_ctx *ctx, hipStream_t s, uint32_t *ptr, size_t words, uint32_t value) {
    if (words == 0) return SCHULZE_OK;
    int64_t blocks = ceil_div((int64_t)(words / 4 + 1), 256);
    if (blocks > (int64_t)ctx->num_cus * 8) blocks = (int64_t)ctx->num_cus * 8;
    if (blocks < 1) blocks = 1;
    SCHULZE_LAUNCH(ctx, K_FILL, s, k_fill_u32<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ptr, words, value));
    return SCHULZE_OK;
}

// ---------------------------------------------------------------- timing

static hipEvent_t take_event(schulze_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timing_begin(schulze_ctx *ctx, int kernel, hipStream_t s, int *token) {
    *token = -1;
    if (!ctx->timing) return;
    PendingTiming p;
    p.name = kernel;
    p.start = take_event(ctx);
    p.stop = take_event(ctx);
    if (!p.start || !p.stop) return;
    (void)hipEventRecord(p.start, s);
    ctx->pending.push_back(p);
    *token = (int)ctx->pending.size() - 1;
}

void timing_end(schulze_ctx *ctx, int token, hipStream_t s) {
    if (token < 0) return;
    (void)hipEventRecord(ctx->pending[token].stop, s);
}

static int drain_timing(schulze_ctx *ctx) {
    int rc = SCHULZE_OK;
    for (auto &p : ctx->pending) {
        if (hipEventSynchronize(p.stop) != hipSuccess) rc = SCHULZE_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            ctx->launches[p.name] += 1;
            ctx->total_ms[p.name] += ms;
        } else {
            rc = SCHULZE_EDEVICE;
        }
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    ctx->pending.clear();
    return rc;
}

extern "C" int schulze_set_closure_schedule(schulze_ctx *ctx, int schedule) {
    if (!ctx || (schedule != SCHULZE_SCHEDULE_AUTO && schedule != SCHULZE_SCHEDULE_PHASED)) return SCHULZE_EINVAL;
    ctx->force_phased = schedule == SCHULZE_SCHEDULE_PHASED;
    return SCHULZE_OK;
}

extern "C" int schulze_set_sparse_count(schulze_ctx *ctx, int mode) {
    if (!ctx || (mode != SCHULZE_SPARSE_BUCKETED && mode != SCHULZE_SPARSE_ATOMIC)) return SCHULZE_EINVAL;
    ctx->legacy_pairs = mode == SCHULZE_SPARSE_ATOMIC;
    return SCHULZE_OK;
}

extern "C" int schulze_set_closure_tile(schulze_ctx *ctx, int tile) {
    if (!ctx || (tile != 0 && tile != 64 && tile != 128)) return SCHULZE_EINVAL;
    ctx->closure_tile = tile;
    return SCHULZE_OK;
}

extern "C" int schulze_set_value_ranking(schulze_ctx *ctx, int enable) {
    if (!ctx) return SCHULZE_EINVAL;
    ctx->value_ranking = enable != 0;
    return SCHULZE_OK;
}

extern "C" int schulze_set_sweep_limits(schulze_ctx *ctx, int64_t spin_limit, int32_t max_sweeps) {
    if (!ctx || spin_limit < 0 || max_sweeps < 0) return SCHULZE_EINVAL;
    ctx->sweep_spin_limit = spin_limit;
    ctx->sweep_max_sweeps = max_sweeps;
    return SCHULZE_OK;
}

extern "C" int schulze_closure_value_bits(schulze_ctx *ctx, void *stream, int32_t *value_bits) {
    if (!ctx || !value_bits) return SCHULZE_EINVAL;
    if (ctx->closure_bits != 0 || !ctx->closure_ranked_flag) {
        *value_bits = ctx->closure_bits;
        return SCHULZE_OK;
    }
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    int32_t ranked = 0;
    if (hipMemcpyAsync(&ranked, ctx->closure_ranked_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SCHULZE_EDEVICE;
    *value_bits = ranked ? 16 : 32;
    return SCHULZE_OK;
}

extern "C" int schulze_set_timing(schulze_ctx *ctx, int enable) {
    if (!ctx) return SCHULZE_EINVAL;
    ctx->timing = enable != 0;
    return SCHULZE_OK;
}

extern "C" int schulze_reset_timing(schulze_ctx *ctx) {
    if (!ctx) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    int rc = drain_timing(ctx);
    ctx->launches.assign(K_NUM_KERNELS, 0);
    ctx->total_ms.assign(K_NUM_KERNELS, 0.0);
    return rc;
}

extern "C" int schulze_kernel_time(schulze_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms) {
    if (!ctx || !kernel || !launches || !total_ms) return SCHULZE_EINVAL;
    if (bind_device(ctx) != SCHULZE_OK) return SCHULZE_EDEVICE;
    int rc = drain_timing(ctx);
    for (int i = 0; i < K_NUM_KERNELS; ++i) {
        if (strcmp(kKernelNames[i], kernel) == 0) {
            *launches = ctx->launches[i];
            *total_ms = ctx->total_ms[i];
            return rc;
        }
    }
    return SCHULZE_EINVAL;
}
