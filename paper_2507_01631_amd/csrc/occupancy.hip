// Coarse occupancy grid and sample culling (the SAT-NGP procedure the paper
// follows during training, Sec. 4.1): every NeRF tile keeps a G^3 grid over
// its [0,1]^3 frame holding a decaying maximum of the density seen at the
// cell centres; samples whose cell is not occupied are removed before the
// field is evaluated.  Empty space then adds no optical depth, so the
// quadrature over the kept intervals is that of the full ray with sigma = 0
// in the culled ones.
//
// Cell of a tile-frame position x: c_a = min(floor(x_a G), G - 1), flattened
// (c_x G + c_y) G + c_z, tile k's grid at offset k G^3; G is a power of two,
// so x_a G is exact.  Occupancy bits: cell c is bit c % 32 of word c / 32.
#include "common.h"
#include "scan.h"

namespace snake {
namespace {

__device__ __forceinline__ int64_t cell_of(const float *p, int G)
{
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = floorf(p[a] * (float)G);
        f = fminf(fmaxf(f, 0.0f), (float)(G - 1));
        c[a] = (int)f;
    }
    return ((int64_t)c[0] * G + c[1]) * G + c[2];
}

__global__ __launch_bounds__(256) void cells_kernel(int G, int K, float *__restrict__ pos, uint8_t *__restrict__ tile)
{
    const int64_t per = (int64_t)G * G * G, total = per * K;
    const float inv = 1.0f / (float)G;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = c / per, r = c - k * per;
        const int i = (int)(r / ((int64_t)G * G)), j = (int)((r / G) % G), l = (int)(r % G);
        pos[3 * c] = ((float)i + 0.5f) * inv;
        pos[3 * c + 1] = ((float)j + 0.5f) * inv;
        pos[3 * c + 2] = ((float)l + 0.5f) * inv;
        if (tile) tile[c] = (uint8_t)k;
    }
}

// Compensated FP32 sums ("float-float": a value and its rounding error),
// about 2^-44 relative over the grid without FP64 arithmetic.
struct FF {
    float hi, lo;
};

__device__ __forceinline__ FF ff_two_sum(float a, float b)
{
    const float s = a + b;
    const float bb = s - a;
    return FF{s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ FF ff_add(FF x, FF y)
{
    const FF s = ff_two_sum(x.hi, y.hi);
    const float lo = s.lo + (x.lo + y.lo);
    const float hi = s.hi + lo;                  // renormalise: |lo| is far below |s.hi|
    return FF{hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ FF ff_wave_sum(FF v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const FF u{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)};
        v = ff_add(v, u);
    }
    return v;
}

// Occupancy update, first half: density = max(decay density, scale sigma)
// for every cell, and each block's compensated sum of the new densities (for
// the mean cap).  The grid is a function of n alone and every block sums its
// cells in a fixed order, so the partial sums are reproducible.
__global__ __launch_bounds__(256) void occ_decay_kernel(const float *__restrict__ sigma, int64_t n, float decay,
                                                        float scale, float *__restrict__ density,
                                                        float2 *__restrict__ partial)
{
    __shared__ FF red[4];
    FF acc{0.0f, 0.0f};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const float d = fmaxf(density[c] * decay, scale * sigma[c]);
        density[c] = d;
        acc = ff_add(acc, FF{d, 0.0f});
    }
    acc = ff_wave_sum(acc);
    if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const FF s = ff_add(ff_add(red[0], red[1]), ff_add(red[2], red[3]));
        partial[blockIdx.x] = make_float2(s.hi, s.lo);
    }
}

// Second half: bit = density > thr, with thr = min(threshold, mean density)
// under the mean cap (every block adds the partial sums in the same order).
// One wavefront writes the two 32-bit words of its 64 cells.
__global__ __launch_bounds__(256) void occ_bits_kernel(const float *__restrict__ density, int64_t n, float threshold,
                                                       int mean_cap, const float2 *__restrict__ partial, int nparts,
                                                       uint32_t *__restrict__ bits)
{
    __shared__ FF red[4];
    __shared__ float thr_s;
    if (mean_cap) {
        FF acc{0.0f, 0.0f};
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc = ff_add(acc, FF{partial[i].x, partial[i].y});
        acc = ff_wave_sum(acc);
        if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const FF s = ff_add(ff_add(red[0], red[1]), ff_add(red[2], red[3]));
            const float mean = (s.hi + s.lo) / (float)n;
            thr_s = fminf(threshold, mean);
        }
    } else if (threadIdx.x == 0) {
        thr_s = threshold;
    }
    __syncthreads();
    const float thr = thr_s;
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); w * 64 < n; w += waves) {
        const int64_t c = w * 64 + lane;
        const bool occ = c < n && density[c] > thr;
        const unsigned long long m = __ballot(occ);
        if (lane == 0) bits[2 * w] = (uint32_t)m;
        if (lane == 32 && w * 64 + 32 < n) bits[2 * w + 1] = (uint32_t)(m >> 32);
    }
}

constexpr int kOccBlocks = 1024;

static unsigned occ_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > kOccBlocks ? kOccBlocks : b));
}

__device__ __forceinline__ bool sample_kept(const float *pos, const uint8_t *tile_id, int64_t s, int G, int K,
                                            const uint32_t *bits, unsigned int *err)
{
    const int k = tile_id ? tile_id[s] : 0;
    if (k >= K) {
        if (err) atomicOr(err, (unsigned)SNAKE_DEVERR_TILE_ID);
        return false;
    }
    const int64_t c = (int64_t)k * G * G * G + cell_of(pos + 3 * s, G);
    return (bits[c >> 5] >> (c & 31)) & 1u;
}

// One wavefront per ray: number of kept samples.
__global__ __launch_bounds__(256) void cull_count_kernel(const int32_t *__restrict__ info, int R,
                                                         const float *__restrict__ pos,
                                                         const uint8_t *__restrict__ tile_id, int G, int K,
                                                         const uint32_t *__restrict__ bits,
                                                         int32_t *__restrict__ counts, unsigned int *err)
{
    const int lane = lane_id();
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < R; r += waves) {
        const int64_t start = info[2 * (int64_t)r];
        const int count = info[2 * (int64_t)r + 1];
        int kept = 0;
        for (int c0 = 0; c0 < count; c0 += 64) {
            const bool k = c0 + lane < count && sample_kept(pos, tile_id, start + c0 + lane, G, K, bits, err);
            kept += __popcll(__ballot(k));
        }
        if (lane == 0) counts[r] = kept;
    }
}

__global__ __launch_bounds__(256) void cull_fill_kernel(
    const int32_t *__restrict__ info, int R, const float *__restrict__ t0, const float *__restrict__ t1,
    const float *__restrict__ pos, const int32_t *__restrict__ ray_id, const uint8_t *__restrict__ tile_id, int G,
    int K, const uint32_t *__restrict__ bits, const int32_t *__restrict__ info_out, int64_t cap,
    float *__restrict__ t0_o, float *__restrict__ t1_o, float *__restrict__ pos_o, int32_t *__restrict__ ray_o,
    uint8_t *__restrict__ tile_o)
{
    const int lane = lane_id();
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < R; r += waves) {
        const int64_t start = info[2 * (int64_t)r];
        const int count = info[2 * (int64_t)r + 1];
        int64_t o = info_out[2 * (int64_t)r];
        for (int c0 = 0; c0 < count; c0 += 64) {
            const int64_t s = start + c0 + lane;
            const bool k = c0 + lane < count && sample_kept(pos, tile_id, s, G, K, bits, nullptr);
            const unsigned long long m = __ballot(k);
            const int64_t d = o + __popcll(m & lt);
            if (k && d < cap) {
                t0_o[d] = t0[s];
                t1_o[d] = t1[s];
                pos_o[3 * d] = pos[3 * s];
                pos_o[3 * d + 1] = pos[3 * s + 1];
                pos_o[3 * d + 2] = pos[3 * s + 2];
                ray_o[d] = ray_id[s];
                if (tile_o) tile_o[d] = tile_id ? tile_id[s] : 0;
            }
            o += __popcll(m);
        }
    }
}

__global__ void set_zero_kernel(int64_t *p) { *p = 0; }

size_t cull_ws_bytes(int32_t R)
{
    const size_t r = (size_t)(R > 0 ? R : 1);
    return ((r * 4 + 255) / 256) * 256 + (size_t)scan::scan_blocks((int64_t)r) * 8 + 256;
}

bool pow2(int G) { return G >= 2 && G <= 1024 && (G & (G - 1)) == 0; }

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

int snake_occupancy_cells(int32_t G, int32_t K, float *pos, uint8_t *tile_id, snake_stream_t stream)
{
    SNAKE_REQUIRE(pow2(G), SNAKE_ERR_INVALID_ARG, "snake_occupancy_cells: G = %d not a power of two in [2, 1024]", G);
    SNAKE_REQUIRE(K >= 1 && K <= 256, SNAKE_ERR_INVALID_ARG, "snake_occupancy_cells: K = %d not in [1, 256]", K);
    SNAKE_NOT_NULL(pos);
    const int64_t total = (int64_t)G * G * G * K;
    cells_kernel<<<grid_for(total, 256, 8), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(G, K, pos, tile_id);
    return launch_status(__func__);
}

size_t snake_occupancy_workspace_bytes(int64_t n_cells)
{
    return n_cells < 0 ? 0 : (size_t)occ_blocks(n_cells) * sizeof(float2);
}

int snake_occupancy_update(const float *sigma, int64_t n_cells, float decay, float sigma_scale, float threshold,
                           uint32_t flags, float *density, uint32_t *bits, void *workspace, size_t workspace_bytes,
                           snake_stream_t stream)
{
    SNAKE_REQUIRE(n_cells >= 0, SNAKE_ERR_INVALID_ARG, "snake_occupancy_update: n_cells < 0");
    SNAKE_REQUIRE(decay >= 0.0f && decay <= 1.0f, SNAKE_ERR_INVALID_ARG, "snake_occupancy_update: decay not in [0, 1]");
    SNAKE_REQUIRE(sigma_scale > 0.0f && sigma_scale <= 3.4e38f, SNAKE_ERR_INVALID_ARG,
                  "snake_occupancy_update: sigma_scale must be positive and finite");
    SNAKE_REQUIRE((flags & ~SNAKE_OCC_MEAN_CAP) == 0u, SNAKE_ERR_INVALID_ARG, "snake_occupancy_update: unknown flags");
    if (n_cells == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(sigma);
    SNAKE_NOT_NULL(density);
    SNAKE_NOT_NULL(bits);
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= snake_occupancy_workspace_bytes(n_cells),
                  SNAKE_ERR_WORKSPACE, "snake_occupancy_update: workspace needs %zu bytes",
                  snake_occupancy_workspace_bytes(n_cells));
    SNAKE_ALIGNED(workspace, 8);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = occ_blocks(n_cells);
    float2 *partial = static_cast<float2 *>(workspace);
    occ_decay_kernel<<<nb, 256, 0, st>>>(sigma, n_cells, decay, sigma_scale, density, partial);
    occ_bits_kernel<<<grid_for(n_cells, 256, 8), 256, 0, st>>>(density, n_cells, threshold,
                                                               (flags & SNAKE_OCC_MEAN_CAP) ? 1 : 0, partial,
                                                               (int)nb, bits);
    return launch_status(__func__);
}

size_t snake_cull_workspace_bytes(int32_t R) { return cull_ws_bytes(R); }

int snake_cull_samples(int32_t G, const uint32_t *bits, int32_t K, int32_t R, const int32_t *packed_info,
                       const float *t0, const float *t1, const float *pos, const int32_t *ray_id,
                       const uint8_t *tile_id, int32_t *packed_info_out, float *t0_out, float *t1_out,
                       float *pos_out, int32_t *ray_id_out, uint8_t *tile_id_out, int64_t cap, int64_t *n_out,
                       void *workspace, size_t workspace_bytes, snake_stream_t stream)
{
    SNAKE_REQUIRE(pow2(G), SNAKE_ERR_INVALID_ARG, "snake_cull_samples: G = %d not a power of two in [2, 1024]", G);
    SNAKE_REQUIRE(K >= 1 && K <= 256, SNAKE_ERR_INVALID_ARG, "snake_cull_samples: K = %d not in [1, 256]", K);
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "snake_cull_samples: R < 0");
    SNAKE_REQUIRE(cap >= 0 && cap <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "snake_cull_samples: cap not in [0, 2^31)");
    SNAKE_NOT_NULL(n_out);
    SNAKE_REQUIRE(K == 1 || tile_id != nullptr, SNAKE_ERR_NULL, "snake_cull_samples: tile_id is NULL with K > 1");
    if (R > 0) {
        SNAKE_NOT_NULL(bits);
        SNAKE_NOT_NULL(packed_info);
        SNAKE_NOT_NULL(t0);
        SNAKE_NOT_NULL(t1);
        SNAKE_NOT_NULL(pos);
        SNAKE_NOT_NULL(ray_id);
        SNAKE_NOT_NULL(packed_info_out);
    }
    if (cap > 0) {
        SNAKE_NOT_NULL(t0_out);
        SNAKE_NOT_NULL(t1_out);
        SNAKE_NOT_NULL(pos_out);
        SNAKE_NOT_NULL(ray_id_out);
    }
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= cull_ws_bytes(R), SNAKE_ERR_WORKSPACE,
                  "snake_cull_samples: workspace needs %zu bytes", cull_ws_bytes(R));
    SNAKE_ALIGNED(workspace, 256);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (R == 0) {
        set_zero_kernel<<<1, 1, 0, st>>>(n_out);
        return launch_status(__func__);
    }
    const size_t r = (size_t)R;
    int32_t *counts = static_cast<int32_t *>(workspace);
    int64_t *bsum = reinterpret_cast<int64_t *>(static_cast<char *>(workspace) + ((r * 4 + 255) / 256) * 256);
    unsigned int *err = device_error_word();
    const unsigned gw = grid_for((int64_t)R * 64, 256, 16);
    cull_count_kernel<<<gw, 256, 0, st>>>(packed_info, R, pos, tile_id, G, K, bits, counts, err);
    scan::launch_scan(counts, R, bsum, packed_info_out, 2, packed_info_out + 1, cap, n_out, err, st);
    cull_fill_kernel<<<gw, 256, 0, st>>>(packed_info, R, t0, t1, pos, ray_id, tile_id, G, K, bits, packed_info_out,
                                         cap, t0_out, t1_out, pos_out, ray_id_out, tile_id_out);
    return launch_status(__func__);
}

}  // extern "C"
