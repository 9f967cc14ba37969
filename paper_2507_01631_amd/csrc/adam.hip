// Adam with bias correction (the I-NGP optimisation strategy, Sec. 4.6),
// FP32 parameters and moments, 4 parameters per lane, HBM-bound (28 B/param).
//
// No FMA contraction in this file: every kernel (one tensor or K tiles, host
// or device step) then rounds the same operations the same way.
#pragma clang fp contract(off)

#include <math.h>

#include "common.h"

namespace snake {
namespace {

struct AdamArgs {
    float lr, b1, b2, eps, l2, c1, c2;   // c1 = 1 - b1^step, c2 = 1 - b2^step
    int zero_grad;
    const int32_t *step_dev;             // step read on the device when set
};

// b^k by binary powering in FP32: the same multiplications, in the same
// order, on the host and on the device, so both give the same bits.
__host__ __device__ inline float pow_int(float b, int k)
{
    float r = 1.0f;
    while (k > 0) {
        if (k & 1) r *= b;
        b *= b;
        k >>= 1;
    }
    return r;
}

__host__ __device__ inline void bias_corrections(AdamArgs &a, int step)
{
    a.c1 = 1.0f - pow_int(a.b1, step);
    a.c2 = 1.0f - pow_int(a.b2, step);
}

__device__ __forceinline__ void adam1(float &p, float &g, float &m, float &v, const AdamArgs &a)
{
    const float gi = g + a.l2 * p;
    m = a.b1 * m + (1.0f - a.b1) * gi;
    v = a.b2 * v + (1.0f - a.b2) * gi * gi;
    const float mh = m / a.c1, vh = v / a.c2;
    p -= a.lr * mh / (sqrtf(vh) + a.eps);
    if (a.zero_grad) g = 0.0f;
}

__global__ __launch_bounds__(256) void adam_kernel(float4 *__restrict__ p, float4 *__restrict__ g,
                                                   float4 *__restrict__ m, float4 *__restrict__ v, int64_t n4,
                                                   float *__restrict__ ps, float *__restrict__ gs,
                                                   float *__restrict__ ms, float *__restrict__ vs, int tail,
                                                   AdamArgs a)
{
    if (a.step_dev) {
        const int step = *a.step_dev;
        bias_corrections(a, step < 1 ? 1 : step);
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        float4 P = p[i], G = g[i], M = m[i], V = v[i];
        adam1(P.x, G.x, M.x, V.x, a);
        adam1(P.y, G.y, M.y, V.y, a);
        adam1(P.z, G.z, M.z, V.z, a);
        adam1(P.w, G.w, M.w, V.w, a);
        p[i] = P;
        m[i] = M;
        v[i] = V;
        if (a.zero_grad) g[i] = G;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < tail) {
        const int k = threadIdx.x;
        float P = ps[k], G = gs[k], M = ms[k], V = vs[k];
        adam1(P, G, M, V, a);
        ps[k] = P;
        ms[k] = M;
        vs[k] = V;
        if (a.zero_grad) gs[k] = G;
    }
}

// K parameter blocks of tile_n floats, block k with the step in step_dev[k]:
// grid (blocks per tile, K), so a block's tile, hence its bias corrections,
// are uniform.
constexpr int kMaxAdamTiles = 64;

__global__ __launch_bounds__(256) void adam_tiles_kernel(float *__restrict__ p, float *__restrict__ g,
                                                         float *__restrict__ m, float *__restrict__ v, int64_t tile_n,
                                                         const int32_t *__restrict__ step_dev, AdamArgs a)
{
    const int k = blockIdx.y;
    const int step = step_dev[k];
    bias_corrections(a, step < 1 ? 1 : step);
    const int64_t base = (int64_t)k * tile_n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tile_n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = base + i;
        float P = p[e], G = g[e], M = m[e], V = v[e];
        adam1(P, G, M, V, a);
        p[e] = P;
        m[e] = M;
        v[e] = V;
        if (a.zero_grad) g[e] = G;
    }
}

__global__ void counter_add_kernel(int32_t *c, int n, int32_t d)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] += d;
}

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

int snake_counter_add(int32_t *counter, int32_t n, int32_t delta, snake_stream_t stream)
{
    SNAKE_REQUIRE(n >= 0 && n <= (1 << 20), SNAKE_ERR_INVALID_ARG, "snake_counter_add: n = %d not in [0, 2^20]", n);
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(counter);
    counter_add_kernel<<<(n + 63) / 64, 64, 0, reinterpret_cast<hipStream_t>(stream)>>>(counter, n, delta);
    return launch_status(__func__);
}

int snake_adam_step(float *p, float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                    int32_t step, const int32_t *step_dev, float l2, uint32_t flags, snake_stream_t stream)
{
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_adam_step: n < 0");
    SNAKE_REQUIRE(step_dev != nullptr || step >= 1, SNAKE_ERR_INVALID_ARG, "snake_adam_step: step = %d < 1",
                  step);
    SNAKE_REQUIRE(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f, SNAKE_ERR_INVALID_ARG,
                  "snake_adam_step: betas must be in [0, 1)");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(p);
    SNAKE_NOT_NULL(g);
    SNAKE_NOT_NULL(m);
    SNAKE_NOT_NULL(v);
    SNAKE_ALIGNED(p, 16);
    SNAKE_ALIGNED(g, 16);
    SNAKE_ALIGNED(m, 16);
    SNAKE_ALIGNED(v, 16);
    AdamArgs a;
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.l2 = l2;
    a.step_dev = step_dev;
    bias_corrections(a, step_dev ? 1 : step);
    a.zero_grad = (flags & SNAKE_ADAM_ZERO_GRAD) ? 1 : 0;
    const int64_t n4 = n / 4;
    const int tail = (int)(n - n4 * 4);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    adam_kernel<<<grid_for(n4 > 0 ? n4 : 1, 256, 8), 256, 0, st>>>(
        reinterpret_cast<float4 *>(p), reinterpret_cast<float4 *>(g), reinterpret_cast<float4 *>(m),
        reinterpret_cast<float4 *>(v), n4, p + n4 * 4, g + n4 * 4, m + n4 * 4, v + n4 * 4, tail, a);
    return launch_status(__func__);
}

int snake_adam_step_tiles(float *p, float *g, float *m, float *v, int64_t tile_n, int32_t K, float lr, float b1,
                          float b2, float eps, const int32_t *step_dev, float l2, uint32_t flags,
                          snake_stream_t stream)
{
    SNAKE_REQUIRE(tile_n >= 0 && K >= 1 && K <= kMaxAdamTiles, SNAKE_ERR_INVALID_ARG,
                  "snake_adam_step_tiles: tile_n = %lld, K = %d (1 <= K <= %d)", (long long)tile_n, K, kMaxAdamTiles);
    SNAKE_REQUIRE(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f, SNAKE_ERR_INVALID_ARG,
                  "snake_adam_step_tiles: betas must be in [0, 1)");
    if (tile_n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(p);
    SNAKE_NOT_NULL(g);
    SNAKE_NOT_NULL(m);
    SNAKE_NOT_NULL(v);
    SNAKE_NOT_NULL(step_dev);
    AdamArgs a;
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.l2 = l2;
    a.step_dev = nullptr;
    a.c1 = a.c2 = 1.0f;
    a.zero_grad = (flags & SNAKE_ADAM_ZERO_GRAD) ? 1 : 0;
    unsigned gx = grid_for(tile_n, 256, 8);
    const unsigned per_tile = (unsigned)((8 * num_cus() + K - 1) / K);
    if (gx > per_tile) gx = per_tile > 0 ? per_tile : 1;
    adam_tiles_kernel<<<dim3(gx, (unsigned)K), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(p, g, m, v, tile_n,
                                                                                                 step_dev, a);
    return launch_status(__func__);
}

}  // extern "C"
