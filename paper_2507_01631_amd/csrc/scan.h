// Device-wide exclusive scan of int32 counts (three launches: per-block
// sums, one-block scan of the sums, per-block apply).  Internal.
#pragma once

#include "common.h"

namespace snake {
namespace scan {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;  // counts per scan block

static __device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *total, int64_t *sh)
{
    // 256 threads = 4 waves; sh holds 4 wave totals
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        int64_t u = __shfl_up(inc, dd, 64);
        if (l >= dd) inc += u;
    }
    if (l == 63) sh[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanBlock / 64; ++i) {
        if (i < w) before += sh[i];
        all += sh[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

static __global__ __launch_bounds__(kScanBlock) void scan_partial_kernel(const int32_t *__restrict__ counts,
                                                                  int64_t R, int64_t *__restrict__ bsum)
{
    __shared__ int64_t sh[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e)
        if (base + e < R) s += counts[base + e];
    int64_t tot;
    block_exclusive_scan(s, &tot, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

static __global__ __launch_bounds__(kScanBlock) void scan_top_kernel(int64_t *__restrict__ bsum, int nb,
                                                              int64_t cap, int64_t *__restrict__ n_out,
                                                              unsigned int *__restrict__ err)
{
    __shared__ int64_t sh[4];
    int64_t carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, &tot, sh);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (n_out) *n_out = carry;
        if (carry > cap && err) atomicOr(err, (unsigned)SNAKE_DEVERR_CAPACITY);
    }
}

// start[r * stride] = exclusive prefix; count_dst[r * stride] = count (if given).
// start and count_dst must not alias counts (the pointers are restrict).
static __global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(const int32_t *__restrict__ counts, int64_t R,
                                                                const int64_t *__restrict__ bsum,
                                                                int32_t *__restrict__ start, int stride,
                                                                int32_t *__restrict__ count_dst)
{
    __shared__ int64_t sh[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        c[e] = (base + e < R) ? counts[base + e] : 0;
        s += c[e];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, &tot, sh) + bsum[blockIdx.x];
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        if (base + e < R) {
            start[(base + e) * stride] = (int32_t)ex;
            if (count_dst) count_dst[(base + e) * stride] = c[e];
        }
        ex += c[e];
    }
}


// Blocks of the scan over n counts.
inline int scan_blocks(int64_t n) { return (int)((n + kScanTile - 1) / kScanTile); }

// Exclusive scan of counts[0..n) into start[i * stride] (and counts into
// count_dst[i * stride] when given); bsum holds scan_blocks(n) int64 values;
// *n_out = total; the capacity bit is raised when total > cap.
inline void launch_scan(const int32_t *counts, int64_t n, int64_t *bsum, int32_t *start, int stride,
                        int32_t *count_dst, int64_t cap, int64_t *n_out, unsigned int *err, hipStream_t st)
{
    const int nb = scan_blocks(n);
    scan_partial_kernel<<<nb, kScanBlock, 0, st>>>(counts, n, bsum);
    scan_top_kernel<<<1, kScanBlock, 0, st>>>(bsum, nb, cap, n_out, err);
    scan_apply_kernel<<<nb, kScanBlock, 0, st>>>(counts, n, bsum, start, stride, count_dst);
}

}  // namespace scan
}  // namespace snake
