// Stable partition of samples by NeRF tile.
//
// While a 2x2 window is loaded (Sec. 4.4) every tile keeps its own networks,
// and a 16-sample matrix tile of the MLP kernels must not mix two of them, so
// the window step reorders its samples tile-major once after sampling.  The
// order inside a tile stays the packed (ray, t) order.
//
// count: per block (contiguous sample range) and bucket, a histogram built
//        from wavefront ballots (one LDS add per wavefront and bucket);
// scan:  bucket-major, then block, so block b's slots in bucket k follow
//        those of blocks < b;
// scatter: per 256-sample chunk, ranks from the same ballots plus the counts
//        of the lower wavefronts, then one cursor bump per bucket.
// Bucket K collects tile ids >= K (flagged as SNAKE_DEVERR_TILE_ID).
#include "common.h"
#include "scan.h"

namespace snake {
namespace {

constexpr int kPartBlocks = 2048;
constexpr int kMaxPartTiles = 16;

__global__ __launch_bounds__(256) void part_count_kernel(const uint8_t *__restrict__ tile_id, int64_t n,
                                                         const int64_t *__restrict__ n_dev, int K,
                                                         int32_t *__restrict__ counts, unsigned int *err)
{
    __shared__ int hist[kMaxPartTiles + 1];
    if (threadIdx.x <= K) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t ne = effective_n(n, n_dev);
    const int64_t s0 = ne * blockIdx.x / gridDim.x, s1 = ne * (blockIdx.x + 1) / gridDim.x;
    const int lane = lane_id();
    for (int64_t base = s0; base < s1; base += blockDim.x) {
        const int64_t s = base + threadIdx.x;
        int k = -1;
        if (s < s1) {
            k = tile_id ? tile_id[s] : 0;
            if (k >= K) {
                if (err) atomicOr(err, (unsigned)SNAKE_DEVERR_TILE_ID);
                k = K;
            }
        }
        for (int b = 0; b <= K; ++b) {
            const int c = __popcll(__ballot(k == b));
            if (lane == 0 && c) atomicAdd(&hist[b], c);
        }
    }
    __syncthreads();
    if (threadIdx.x <= K) counts[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(256) void part_scatter_kernel(
    const uint8_t *__restrict__ tile_id, const float *__restrict__ pos, const int32_t *__restrict__ ray_id,
    int64_t n, const int64_t *__restrict__ n_dev, int K, const int32_t *__restrict__ offs,
    int32_t *__restrict__ perm, int32_t *__restrict__ inv, float *__restrict__ pos_out,
    uint8_t *__restrict__ tile_out, int32_t *__restrict__ ray_out)
{
    __shared__ int cursor[kMaxPartTiles + 1];
    __shared__ int wcnt[4][kMaxPartTiles + 1];
    if (threadIdx.x <= K) cursor[threadIdx.x] = offs[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    __syncthreads();
    const int64_t ne = effective_n(n, n_dev);
    const int64_t s0 = ne * blockIdx.x / gridDim.x, s1 = ne * (blockIdx.x + 1) / gridDim.x;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = s0; base < s1; base += blockDim.x) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < s1;
        int k = -1;
        if (valid) {
            k = tile_id ? tile_id[s] : 0;
            k = k < K ? k : K;
        }
        int rank = 0;
        for (int b = 0; b <= K; ++b) {
            const unsigned long long m = __ballot(k == b);
            if (k == b) rank = __popcll(m & lt);
            if (lane == 0) wcnt[wv][b] = __popcll(m);
        }
        __syncthreads();
        int64_t j = -1;
        if (valid) {
            int before = 0;
            for (int w = 0; w < wv; ++w) before += wcnt[w][k];
            j = (int64_t)cursor[k] + before + rank;
        }
        __syncthreads();
        if (threadIdx.x <= K) {
            int t = 0;
            for (int w = 0; w < 4; ++w) t += wcnt[w][threadIdx.x];
            cursor[threadIdx.x] += t;
        }
        if (valid && j >= 0 && j < ne) {
            perm[j] = (int32_t)s;
            if (inv) inv[s] = (int32_t)j;
            if (pos_out) {
                pos_out[3 * j] = pos[3 * s];
                pos_out[3 * j + 1] = pos[3 * s + 1];
                pos_out[3 * j + 2] = pos[3 * s + 2];
            }
            if (tile_out) tile_out[j] = tile_id ? tile_id[s] : 0;
            if (ray_out) ray_out[j] = ray_id[s];
        }
        __syncthreads();
    }
}

__global__ void part_starts_kernel(const int32_t *__restrict__ offs, int G, int K, const int64_t *__restrict__ total,
                                   int64_t *__restrict__ tile_start)
{
    const int k = threadIdx.x;
    if (k <= K) tile_start[k] = offs[(int64_t)k * G];
    if (k == 0) tile_start[K + 1] = *total;
}

size_t part_ws_bytes(int K)
{
    const int64_t nc = (int64_t)(K + 1) * kPartBlocks;
    const size_t a = ((size_t)nc * 4 + 255) / 256 * 256;
    return 2 * a + (size_t)scan::scan_blocks(nc) * 8 + 256 + 256;
}

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

size_t snake_tile_partition_workspace_bytes(int32_t K)
{
    if (K < 1 || K > kMaxPartTiles) return 0;
    return part_ws_bytes(K);
}

int snake_tile_partition(const uint8_t *tile_id, const float *pos, const int32_t *ray_id, int64_t n,
                         const int64_t *n_dev, int32_t K, int32_t *perm, int32_t *inv, int64_t *tile_start,
                         float *pos_out, uint8_t *tile_out, int32_t *ray_out, void *workspace,
                         size_t workspace_bytes, snake_stream_t stream)
{
    SNAKE_REQUIRE(K >= 1 && K <= kMaxPartTiles, SNAKE_ERR_INVALID_ARG,
                  "snake_tile_partition: K = %d not in [1, %d]", K, kMaxPartTiles);
    SNAKE_REQUIRE(n >= 0 && n <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "snake_tile_partition: n not in [0, 2^31)");
    SNAKE_REQUIRE(K == 1 || tile_id != nullptr, SNAKE_ERR_NULL, "snake_tile_partition: tile_id is NULL with K > 1");
    SNAKE_NOT_NULL(tile_start);
    if (n > 0) SNAKE_NOT_NULL(perm);
    SNAKE_REQUIRE(pos_out == nullptr || pos != nullptr, SNAKE_ERR_NULL, "snake_tile_partition: pos is NULL");
    SNAKE_REQUIRE(ray_out == nullptr || ray_id != nullptr, SNAKE_ERR_NULL, "snake_tile_partition: ray_id is NULL");
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= part_ws_bytes(K), SNAKE_ERR_WORKSPACE,
                  "snake_tile_partition: workspace needs %zu bytes", part_ws_bytes(K));
    SNAKE_ALIGNED(workspace, 256);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t nc = (int64_t)(K + 1) * kPartBlocks;
    const size_t a = ((size_t)nc * 4 + 255) / 256 * 256;
    char *p = static_cast<char *>(workspace);
    int32_t *counts = reinterpret_cast<int32_t *>(p);
    int32_t *offs = reinterpret_cast<int32_t *>(p + a);
    int64_t *bsum = reinterpret_cast<int64_t *>(p + 2 * a);
    int64_t *total = reinterpret_cast<int64_t *>(p + 2 * a + (size_t)scan::scan_blocks(nc) * 8 + 256);
    unsigned int *err = device_error_word();
    part_count_kernel<<<kPartBlocks, 256, 0, st>>>(tile_id, n, n_dev, K, counts, err);
    scan::launch_scan(counts, nc, bsum, offs, 1, nullptr, n, total, err, st);
    part_scatter_kernel<<<kPartBlocks, 256, 0, st>>>(tile_id, pos, ray_id, n, n_dev, K, offs, perm, inv, pos_out,
                                                     tile_out, ray_out);
    part_starts_kernel<<<1, 64, 0, st>>>(offs, kPartBlocks, K, total, tile_start);
    return launch_status(__func__);
}

}  // extern "C"
