// Winners and ranking from the closure p (Section 2.1): y beats x iff
// p[y][x] > p[x][y]; x is a Schulze winner iff nobody beats it; the ranking
// orders candidates by how many candidates beat them, then by id.
#include "internal.h"
#include "tile_io.h"

namespace {

// beaten_by[x] += #{y : p[y][x] > p[x][y]} over one pair of 64 x 64 blocks
// of candidates (X, Y), X <= Y: both directions need the same two tiles of
// p, so p is read once.
template <typename E>
__global__ __launch_bounds__(256) void k_beaten_by(const E *__restrict__ p, int64_t ldp, int32_t m,
                                                   int32_t *__restrict__ beaten, int vec) {
    __shared__ E py[64][65];  // py[a][b] = p[Y0 + a][X0 + b]
    __shared__ E px[64][65];  // px[a][b] = p[X0 + a][Y0 + b]
    if (blockIdx.x > blockIdx.y) return;
    const int32_t X0 = blockIdx.x * 64, Y0 = blockIdx.y * 64;
    tio::load<E>(py, p, ldp, Y0, X0, m, m, vec != 0);
    tio::load<E>(px, p, ldp, X0, Y0, m, m, vec != 0);
    __syncthreads();
    const int l = threadIdx.x & 63, part = threadIdx.x >> 6;
    int32_t cx = 0, cy = 0;
    for (int o = part * 16; o < part * 16 + 16; ++o) {
        cx += py[o][l] > px[l][o] ? 1 : 0;  // y = Y0 + o beats x = X0 + l
        cy += px[o][l] > py[l][o] ? 1 : 0;  // x = X0 + o beats y = Y0 + l
    }
    if (cx && X0 + l < m) atomicAdd(&beaten[X0 + l], cx);
    if (X0 != Y0 && cy && Y0 + l < m) atomicAdd(&beaten[Y0 + l], cy);
}

__global__ __launch_bounds__(256) void k_winners(const int32_t *__restrict__ beaten, int32_t m,
                                                 uint8_t *__restrict__ is_winner, int32_t *__restrict__ n_winners) {
    const int32_t x = blockIdx.x * 256 + threadIdx.x;
    const bool w = x < m && beaten[x] == 0;
    if (x < m) is_winner[x] = w ? 1 : 0;
    if (n_winners) {
        const uint64_t b = __ballot(w);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(n_winners, (int32_t)__popcll(b));
    }
}

// order[rank(x)] = x with rank(x) = #{y : (beaten[y], y) < (beaten[x], x)}.
// Keys beaten*m + id are distinct and fit 32 bits for m <= 65535.  A
// workgroup takes RS_X candidates; its RS_G wavefronts count over
// interleaved shares of the keys (staged in LDS RS_CHUNK at a time, each
// read a broadcast) and the shares are summed in LDS.  (One thread per
// candidate over every key left most of the chip idle.)
constexpr int RS_X = 64;
constexpr int RS_G = 16;
constexpr int RS_CHUNK = 4096;
__global__ __launch_bounds__(64 * RS_G) void k_rank_sort(const int32_t *__restrict__ beaten, int32_t m,
                                                         int32_t *__restrict__ order) {
    __shared__ uint32_t keys[RS_CHUNK];
    __shared__ int32_t part[RS_G][RS_X];
    const int xl = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int32_t x = blockIdx.x * RS_X + xl;
    auto key = [&](int32_t y) { return (uint32_t)beaten[y] * (uint32_t)m + (uint32_t)y; };
    const uint32_t kx = x < m ? key(x) : 0xFFFFFFFFu;
    int32_t rank = 0;
    for (int32_t y0 = 0; y0 < m; y0 += RS_CHUNK) {
        __syncthreads();
        for (int i = threadIdx.x; i < RS_CHUNK; i += 64 * RS_G) keys[i] = y0 + i < m ? key(y0 + i) : 0xFFFFFFFFu;
        __syncthreads();
        const int lim = min(RS_CHUNK, m - y0);
        for (int i = grp; i < lim; i += RS_G) rank += keys[i] < kx ? 1 : 0;
    }
    part[grp][xl] = rank;
    __syncthreads();
    if (grp == 0 && x < m) {
        int32_t r = 0;
        for (int g = 0; g < RS_G; ++g) r += part[g][xl];
        order[r] = x;
    }
}

template <typename E>
int beaten_by(schulze_ctx *ctx, hipStream_t s, const E *p, int64_t ldp, int32_t m, int32_t *beaten) {
    int rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(beaten), (size_t)m, 0u);
    if (rc != SCHULZE_OK) return rc;
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(m, 64));
    SCHULZE_LAUNCH(ctx, K_BEATEN_BY, s, k_beaten_by<E><<<grid, dim3(256), 0, s>>>(p, ldp, m, beaten,
                                                                                tio::vec_ok<E>(p, ldp) ? 1 : 0));
    return SCHULZE_OK;
}

int beaten_any(schulze_ctx *ctx, hipStream_t s, const void *p, int64_t ldp, int32_t m, int dtype,
               int32_t *beaten) {
    if (dtype == SCHULZE_U16) return beaten_by(ctx, s, static_cast<const uint16_t *>(p), ldp, m, beaten);
    return beaten_by(ctx, s, static_cast<const int32_t *>(p), ldp, m, beaten);
}

int check_args(schulze_ctx *ctx, const void *p, int64_t ldp, int32_t m, int dtype) {
    if (!ctx || !p) return SCHULZE_EINVAL;
    if (m < 1 || ldp < m) return SCHULZE_EINVAL;
    if (dtype != SCHULZE_U16 && dtype != SCHULZE_I32) return SCHULZE_EINVAL;
    if (m > 65535) return SCHULZE_EUNSUPPORTED;
    return bind_device(ctx);
}

}  // namespace

extern "C" int schulze_winners(schulze_ctx *ctx, void *stream, const void *p, int64_t ldp, int32_t m, int dtype,
                               uint8_t *is_winner, int32_t *n_winners) {
    int rc = check_args(ctx, p, ldp, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (!is_winner) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ws_reserve(ctx, WS_RANK, sizeof(int32_t) * (size_t)m)) != SCHULZE_OK) return rc;
    int32_t *beaten = static_cast<int32_t *>(ctx->ws[WS_RANK]);
    if ((rc = beaten_any(ctx, s, p, ldp, m, dtype, beaten)) != SCHULZE_OK) return rc;
    if (n_winners && (rc = fill_u32(ctx, s, reinterpret_cast<uint32_t *>(n_winners), 1, 0u)) != SCHULZE_OK)
        return rc;
    SCHULZE_LAUNCH(ctx, K_WINNERS, s,
                   k_winners<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s>>>(beaten, m, is_winner, n_winners));
    return SCHULZE_OK;
}

extern "C" int schulze_ranking(schulze_ctx *ctx, void *stream, const void *p, int64_t ldp, int32_t m, int dtype,
                               int32_t *order, int32_t *beaten_by_out) {
    int rc = check_args(ctx, p, ldp, m, dtype);
    if (rc != SCHULZE_OK) return rc;
    if (!order) return SCHULZE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int32_t *beaten = beaten_by_out;
    if (!beaten) {
        if ((rc = ws_reserve(ctx, WS_RANK, sizeof(int32_t) * (size_t)m)) != SCHULZE_OK) return rc;
        beaten = static_cast<int32_t *>(ctx->ws[WS_RANK]);
    }
    if ((rc = beaten_any(ctx, s, p, ldp, m, dtype, beaten)) != SCHULZE_OK) return rc;
    SCHULZE_LAUNCH(ctx, K_RANK_SORT, s,
                   k_rank_sort<<<dim3((unsigned)ceil_div(m, RS_X)), dim3(64 * RS_G), 0, s>>>(beaten, m, order));
    return SCHULZE_OK;
}
