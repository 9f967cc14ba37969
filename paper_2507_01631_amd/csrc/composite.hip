// Volume rendering (the unmodified NeRF quadrature, Sec. 2.2 / 4.5), the
// colour-consistency MSE loss (Sec. 4.4), and their adjoint.
//
// One wavefront per ray, one lane per sample, 64-sample chunks with a carry.
// An optional sample map redirects the per-sample values (sigma, rgb and the
// adjoints): the window step keeps them in tile-partitioned order while t0,
// t1 and packed_info stay in ray order.
// Transmittance T_i = prod_{j<i} exp(-s_j) is taken in the log domain: an
// exclusive wave64 prefix sum of the optical depths s_j = sigma_j delta_j,
// then one exp per sample; alpha_i = -expm1(-s_i) keeps full relative
// precision for thin samples.
#include <math.h>

#include "common.h"

namespace snake {
namespace {

constexpr int kWaves = 4;   // wavefronts per 256-thread block

struct SampleVals {
    float s, w, T, mid, c[3];
    bool valid;
};

// Per-sample quantities of chunk [c0, c0+64) of a ray with `count` samples
// and optical depth `carry` accumulated before the chunk.
__device__ __forceinline__ SampleVals chunk_vals(const float *sigma, const float *rgb, const float *t0,
                                                 const float *t1, const int32_t *map, int64_t start, int count,
                                                 int c0, float carry, float &chunk_depth_sum, float &incl)
{
    const int lane = lane_id();
    SampleVals v;
    const int k = c0 + lane;
    v.valid = k < count;
    float s = 0.0f, a0 = 0.0f, a1 = 0.0f;
    v.c[0] = v.c[1] = v.c[2] = 0.0f;
    if (v.valid) {
        const int64_t idx = start + k;
        const int64_t m = map ? (int64_t)map[idx] : idx;
        a0 = t0[idx];
        a1 = t1[idx];
        s = sigma[m] * (a1 - a0);
        v.c[0] = rgb[3 * m];
        v.c[1] = rgb[3 * m + 1];
        v.c[2] = rgb[3 * m + 2];
    }
    incl = wave_inclusive_sum(s);
    // exclusive prefix = the previous lane's inclusive one (no subtraction,
    // which would cancel when s is large)
    float excl = __shfl_up(incl, 1, 64);
    excl = lane == 0 ? 0.0f : excl;
    v.s = s;
    v.T = expf(-(carry + excl));
    v.w = v.T * (-expm1f(-s));
    v.mid = 0.5f * (a0 + a1);
    chunk_depth_sum = __shfl(incl, 63, 64);
    return v;
}

// Number of leading samples of the chunk that survive early stop (64 if all).
__device__ __forceinline__ int first_dead(const SampleVals &v, float thr)
{
    const unsigned long long dead = __ballot(v.valid && thr > 0.0f && v.T < thr);
    return dead ? __ffsll((long long)dead) - 1 : 64;
}

__global__ __launch_bounds__(256) void composite_fwd_kernel(
    const float *__restrict__ sigma, const float *__restrict__ rgb, const float *__restrict__ t0,
    const float *__restrict__ t1, const int32_t *__restrict__ info, int R, const int32_t *__restrict__ map,
    float thr,
    float *__restrict__ rgb_out, float *__restrict__ opacity, float *__restrict__ depth,
    int32_t *__restrict__ n_alive)
{
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int r = blockIdx.x * kWaves + wv; r < R; r += gridDim.x * kWaves) {
        const int64_t start = info[2 * (int64_t)r];
        const int count = info[2 * (int64_t)r + 1];
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, acc = 0.f, dep = 0.f, carry = 0.f;
        int kept = 0;
        for (int c0 = 0; c0 < count; c0 += 64) {
            float tot, incl;
            SampleVals v = chunk_vals(sigma, rgb, t0, t1, map, start, count, c0, carry, tot, incl);
            const int fd = first_dead(v, thr);
            const bool alive = v.valid && lane < fd;
            if (alive) {
                C0 += v.w * v.c[0];
                C1 += v.w * v.c[1];
                C2 += v.w * v.c[2];
                acc += v.w;
                dep += v.w * v.mid;
            }
            const int nvalid = count - c0 < 64 ? count - c0 : 64;
            kept += fd < nvalid ? fd : nvalid;
            carry += tot;
            if (fd < 64) break;
        }
        C0 = wave_sum(C0);
        C1 = wave_sum(C1);
        C2 = wave_sum(C2);
        acc = wave_sum(acc);
        dep = wave_sum(dep);
        if (lane == 0) {
            rgb_out[3 * (int64_t)r] = C0;
            rgb_out[3 * (int64_t)r + 1] = C1;
            rgb_out[3 * (int64_t)r + 2] = C2;
            if (opacity) opacity[r] = acc;
            if (depth) depth[r] = dep;
            if (n_alive) n_alive[r] = kept;
        }
    }
}

// *loss += loss_scale * sum_r sum_ch (rgb_out - target)^2, by one block in a
// fixed order (each thread a compensated sum over a fixed stride of rays,
// then a fixed tree), so the loss has the same bits on every run.
constexpr int kLossThreads = 1024;

__global__ __launch_bounds__(kLossThreads) void loss_kernel(const float *__restrict__ rgb_out,
                                                            const float *__restrict__ target, int R, float loss_scale,
                                                            float *__restrict__ loss)
{
    __shared__ float red[kLossThreads / 64];
    float s = 0.0f, comp = 0.0f;                 // Kahan sum of this thread's rays
    // rays r = tid, tid + kLossThreads, ... in that order; kLossU of them
    // loaded at once (a ray past R re-reads ray R - 1 and is not added), so
    // the loads overlap instead of each waiting for the one before
    constexpr int kLossU = 8;
    for (int r0 = threadIdx.x; r0 < R; r0 += kLossU * kLossThreads) {
        float o[kLossU][3], g[kLossU][3];
#pragma unroll
        for (int u = 0; u < kLossU; ++u) {
            const int r = r0 + u * kLossThreads < R ? r0 + u * kLossThreads : R - 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o[u][c] = rgb_out[3 * (int64_t)r + c];
                g[u][c] = target[3 * (int64_t)r + c];
            }
        }
        // every load issued before any is used (the selects below keep the
        // compiler from moving a load into a branch of its own)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kLossU; ++u) {
            const bool ok = r0 + u * kLossThreads < R;
            const float e0 = o[u][0] - g[u][0], e1 = o[u][1] - g[u][1], e2 = o[u][2] - g[u][2];
            const float y = (e0 * e0 + e1 * e1 + e2 * e2) - comp;
            const float t = s + y;
            const float c = (t - s) - y;
            s = ok ? t : s;
            comp = ok ? c : comp;
        }
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
        for (int i = 0; i < kLossThreads / 64; ++i) tot += red[i];
        *loss += loss_scale * tot;
    }
}

__global__ __launch_bounds__(256) void composite_bwd_kernel(
    const float *__restrict__ sigma, const float *__restrict__ rgb, const float *__restrict__ t0,
    const float *__restrict__ t1, const int32_t *__restrict__ info, int R, const int32_t *__restrict__ map,
    const int32_t *__restrict__ n_alive,
    const float *__restrict__ target, float loss_scale, float *__restrict__ dsigma, float *__restrict__ drgb)
{
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int r = blockIdx.x * kWaves + wv; r < R; r += gridDim.x * kWaves) {
        const int64_t start = info[2 * (int64_t)r];
        const int count = info[2 * (int64_t)r + 1];
        int kept = count;
        if (n_alive) {
            const int a = n_alive[r];
            kept = a < 0 ? 0 : (a < count ? a : count);
        }
        // pass 1: the ray's colour over the kept samples
        float C[3] = {0.f, 0.f, 0.f}, carry = 0.f;
        for (int c0 = 0; c0 < kept; c0 += 64) {
            float tot, incl;
            SampleVals v = chunk_vals(sigma, rgb, t0, t1, map, start, kept, c0, carry, tot, incl);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) C[ch] += v.w * v.c[ch];
            carry += tot;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) C[ch] = wave_sum(C[ch]);
        float g[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) g[ch] = 2.0f * loss_scale * (C[ch] - target[3 * (int64_t)r + ch]);
        // pass 2: per-sample adjoints; A = running inclusive sum of w c
        float A[3] = {0.f, 0.f, 0.f};
        carry = 0.f;
        for (int c0 = 0; c0 < count; c0 += 64) {
            const int64_t idx = start + c0 + lane;
            const int64_t m = (c0 + lane < count) ? (map ? (int64_t)map[idx] : idx) : 0;
            if (c0 >= kept) {
                if (c0 + lane < count) {
                    dsigma[m] = 0.f;
                    drgb[3 * m] = drgb[3 * m + 1] = drgb[3 * m + 2] = 0.f;
                }
                continue;
            }
            float tot, incl;
            SampleVals v = chunk_vals(sigma, rgb, t0, t1, map, start, kept, c0, carry, tot, incl);
            const float Tn = expf(-(carry + incl));
            float Ai[3], ds = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float wc = v.w * v.c[ch];
                Ai[ch] = A[ch] + wave_inclusive_sum(wc);
                ds += g[ch] * (Tn * v.c[ch] - (C[ch] - Ai[ch]));
                A[ch] += __shfl(Ai[ch] - A[ch], 63, 64);
            }
            if (c0 + lane < count) {
                if (v.valid) {
                    const float delta = t1[idx] - t0[idx];
                    dsigma[m] = delta * ds;
                    drgb[3 * m] = v.w * g[0];
                    drgb[3 * m + 1] = v.w * g[1];
                    drgb[3 * m + 2] = v.w * g[2];
                } else {
                    dsigma[m] = 0.f;
                    drgb[3 * m] = drgb[3 * m + 1] = drgb[3 * m + 2] = 0.f;
                }
            }
            carry += tot;
        }
    }
}

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

int snake_composite_fwd(const float *sigma, const float *rgb, const float *t0, const float *t1,
                        const int32_t *packed_info, int32_t R, const int32_t *sample_map, float early_stop_T,
                        const float *target, float loss_scale, float *rgb_out, float *opacity, float *depth,
                        int32_t *n_alive, float *loss, snake_stream_t stream)
{
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "snake_composite_fwd: R < 0");
    SNAKE_REQUIRE(early_stop_T >= 0.0f && early_stop_T < 1.0f, SNAKE_ERR_INVALID_ARG,
                  "snake_composite_fwd: early_stop_T = %g not in [0, 1)", (double)early_stop_T);
    if (R == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(sigma);
    SNAKE_NOT_NULL(rgb);
    SNAKE_NOT_NULL(t0);
    SNAKE_NOT_NULL(t1);
    SNAKE_NOT_NULL(packed_info);
    SNAKE_NOT_NULL(rgb_out);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    composite_fwd_kernel<<<grid_for((int64_t)R * 64, 256, tune(SNAKE_TUNE_COMPOSITE_BLOCKS_PER_CU)), 256, 0, st>>>(
        sigma, rgb, t0, t1, packed_info, R, sample_map, early_stop_T, rgb_out, opacity, depth, n_alive);
    if (target && loss) loss_kernel<<<1, kLossThreads, 0, st>>>(rgb_out, target, R, loss_scale, loss);
    return launch_status(__func__);
}

int snake_composite_bwd(const float *sigma, const float *rgb, const float *t0, const float *t1,
                        const int32_t *packed_info, int32_t R, const int32_t *sample_map, const int32_t *n_alive,
                        const float *target, float loss_scale, float *dsigma, float *drgb, snake_stream_t stream)
{
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "snake_composite_bwd: R < 0");
    if (R == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(sigma);
    SNAKE_NOT_NULL(rgb);
    SNAKE_NOT_NULL(t0);
    SNAKE_NOT_NULL(t1);
    SNAKE_NOT_NULL(packed_info);
    SNAKE_NOT_NULL(target);
    SNAKE_NOT_NULL(dsigma);
    SNAKE_NOT_NULL(drgb);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    composite_bwd_kernel<<<grid_for((int64_t)R * 64, 256, tune(SNAKE_TUNE_COMPOSITE_BLOCKS_PER_CU)), 256, 0, st>>>(
        sigma, rgb, t0, t1, packed_info, R, sample_map, n_alive, target, loss_scale, dsigma, drgb);
    return launch_status(__func__);
}

}  // extern "C"
