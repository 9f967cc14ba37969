// Multiresolution hash encoding, forward gather and adjoint scatter (Sec. 4.1;
// the NGP representation the paper adopts).
//
// Work order is level-major: the grid-stride loop walks (level, 256-sample
// chunk) units with the level as the slow index, so at any moment the chip
// gathers from one or two levels' slices of the table (T*F*4 bytes each) and
// those stay resident in L2 instead of the whole table competing for it.
// Features are stored level-major [L][n][F] so each level reads/writes
// coalesced.
//
// FMA contraction is off in this file: the cell weight w = fl32(x N) - c must
// use the rounded product, which a fused multiply-subtract would skip.  The
// blend's fused multiply-adds are written out explicitly.
#pragma clang fp contract(off)

#include "common.h"

namespace snake {
namespace {

struct Grid {
    int L;
    int log2T;
    uint32_t mask;        // T - 1
    uint32_t dense_bits;  // bit l set: level l uses dense indexing
    int32_t res[SNAKE_MAX_LEVELS];
};

// Cell of x at resolution N: p = fl32(x N), c = min(floor p, N-1), w = p - c (exact).
__device__ __forceinline__ void cell(float x, int N, uint32_t &c, float &w)
{
    float p = x * (float)N;
    float f = floorf(p);
    f = fminf(f, (float)(N - 1));
    f = fmaxf(f, 0.0f);
    c = (uint32_t)f;
    w = p - f;
}

__device__ __forceinline__ void corners(const Grid &g, int l, const float x[3], uint32_t idx[8],
                                        float wt[8])
{
    const int N = g.res[l];
    uint32_t c[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cell(x[a], N, c[a], w[a]);
    const bool dense = (g.dense_bits >> l) & 1u;
    const uint32_t side = (uint32_t)N + 1u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t i = c[0] + (q & 1), j = c[1] + ((q >> 1) & 1), k = c[2] + ((q >> 2) & 1);
        idx[q] = dense ? i + j * side + k * side * side
                       : ((i * 1u) ^ (j * 2654435761u) ^ (k * 805459861u)) & g.mask;
        const float wx = (q & 1) ? w[0] : 1.0f - w[0];
        const float wy = ((q >> 1) & 1) ? w[1] : 1.0f - w[1];
        const float wz = ((q >> 2) & 1) ? w[2] : 1.0f - w[2];
        wt[q] = (wx * wy) * wz;
    }
}

template <int F>
struct Vec;
template <>
struct Vec<1> {
    typedef float T;
    __device__ static float get(const T &v, int) { return v; }
};
template <>
struct Vec<2> {
    typedef float2 T;
    __device__ static float get(const T &v, int f) { return f ? v.y : v.x; }
};
template <>
struct Vec<4> {
    typedef float4 T;
    __device__ static float get(const T &v, int f) { return f == 0 ? v.x : f == 1 ? v.y : f == 2 ? v.z : v.w; }
};

__device__ __forceinline__ void store_feat(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_feat(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }

template <int F, typename OutT>
__global__ __launch_bounds__(256) void hashgrid_fwd_kernel(Grid g, const float *__restrict__ table,
                                                           const float *__restrict__ pos,
                                                           const uint8_t *__restrict__ tile_id,
                                                           const int32_t *__restrict__ sidx, int64_t n,
                                                           const int64_t *__restrict__ n_dev,
                                                           OutT *__restrict__ feat,
                                                           uint32_t *__restrict__ idx_dbg)
{
    typedef typename Vec<F>::T VT;
    const int64_t ne = effective_n(n, n_dev);
    const int64_t chunks = (ne + 255) / 256;
    const int64_t units = chunks * g.L;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int l = (int)(u / chunks);
        const int64_t s = (u - (int64_t)l * chunks) * 256 + threadIdx.x;
        if (s >= ne) continue;
        const int64_t si = sidx ? sidx[s] : s;
        const float x[3] = {pos[3 * si], pos[3 * si + 1], pos[3 * si + 2]};
        const int64_t tile = tile_id ? tile_id[si] : 0;
        uint32_t idx[8];
        float wt[8];
        corners(g, l, x, idx, wt);
        const VT *lev = reinterpret_cast<const VT *>(table + ((tile * g.L + l) << g.log2T) * F);
        VT v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = lev[idx[q]];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = fmaf(wt[q], Vec<F>::get(v[q], f), acc);
            store_feat(feat + ((int64_t)l * n + s) * F + f, acc);
        }
        if (idx_dbg) {
#pragma unroll
            for (int q = 0; q < 8; ++q) idx_dbg[(s * g.L + l) * 8 + q] = idx[q];
        }
    }
}

template <int F>
__global__ __launch_bounds__(256) void hashgrid_bwd_kernel(Grid g, const float *__restrict__ pos,
                                                           const uint8_t *__restrict__ tile_id,
                                                           const int32_t *__restrict__ sidx, int64_t n,
                                                           const int64_t *__restrict__ n_dev,
                                                           const float *__restrict__ dfeat,
                                                           float *__restrict__ dtable)
{
    typedef typename Vec<F>::T VT;
    const int64_t ne = effective_n(n, n_dev);
    const int64_t chunks = (ne + 255) / 256;
    const int64_t units = chunks * g.L;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int l = (int)(u / chunks);
        const int64_t s = (u - (int64_t)l * chunks) * 256 + threadIdx.x;
        if (s >= ne) continue;
        const VT gv = *reinterpret_cast<const VT *>(dfeat + ((int64_t)l * n + s) * F);
        bool any = false;
#pragma unroll
        for (int f = 0; f < F; ++f) any |= Vec<F>::get(gv, f) != 0.0f;
        if (!any) continue;
        const int64_t si = sidx ? sidx[s] : s;
        const float x[3] = {pos[3 * si], pos[3 * si + 1], pos[3 * si + 2]};
        const int64_t tile = tile_id ? tile_id[si] : 0;
        uint32_t idx[8];
        float wt[8];
        corners(g, l, x, idx, wt);
        float *lev = dtable + ((tile * g.L + l) << g.log2T) * F;
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int f = 0; f < F; ++f)
                unsafeAtomicAdd(lev + (int64_t)idx[q] * F + f, wt[q] * Vec<F>::get(gv, f));
    }
}

int make_grid(const snake_grid_desc *d, Grid &g, const char *fn)
{
    SNAKE_REQUIRE(d != nullptr, SNAKE_ERR_NULL, "%s: grid descriptor is NULL", fn);
    SNAKE_REQUIRE(d->n_levels >= 1 && d->n_levels <= SNAKE_MAX_LEVELS, SNAKE_ERR_INVALID_ARG,
                  "%s: n_levels = %d not in [1, %d]", fn, d->n_levels, SNAKE_MAX_LEVELS);
    SNAKE_REQUIRE(d->n_features == 1 || d->n_features == 2 || d->n_features == 4, SNAKE_ERR_UNSUPPORTED,
                  "%s: n_features = %d not in {1, 2, 4}", fn, d->n_features);
    SNAKE_REQUIRE(d->log2_table >= 4 && d->log2_table <= 24, SNAKE_ERR_INVALID_ARG,
                  "%s: log2_table = %d not in [4, 24]", fn, d->log2_table);
    SNAKE_REQUIRE(d->feat_dtype == SNAKE_F32 || d->feat_dtype == SNAKE_BF16, SNAKE_ERR_INVALID_ARG,
                  "%s: bad feat_dtype %d", fn, d->feat_dtype);
    g.L = d->n_levels;
    g.log2T = d->log2_table;
    g.mask = (uint32_t)((1ull << d->log2_table) - 1);
    g.dense_bits = 0;
    const uint64_t T = 1ull << d->log2_table;
    for (int l = 0; l < g.L; ++l) {
        const int N = d->resolution[l];
        SNAKE_REQUIRE(N >= 1 && N <= (1 << 20), SNAKE_ERR_INVALID_ARG,
                      "%s: resolution[%d] = %d not in [1, 2^20]", fn, l, N);
        g.res[l] = N;
        const uint64_t side = (uint64_t)N + 1;
        if (!(d->flags & SNAKE_GRID_ALWAYS_HASH) && side * side * side <= T) g.dense_bits |= 1u << l;
    }
    for (int l = g.L; l < SNAKE_MAX_LEVELS; ++l) g.res[l] = 1;
    return SNAKE_OK;
}

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

int snake_hashgrid_fwd(const snake_grid_desc *gd, const float *table, const float *pos,
                       const uint8_t *tile_id, const int32_t *sample_idx, int64_t n,
                       const int64_t *n_dev, void *feat, uint32_t *idx_dbg, snake_stream_t stream)
{
    Grid g;
    int rc = make_grid(gd, g, __func__);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_hashgrid_fwd: n < 0");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(table);
    SNAKE_NOT_NULL(pos);
    SNAKE_NOT_NULL(feat);
    SNAKE_ALIGNED(table, 16);
    const int F = gd->n_features;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned grid = grid_for(n * g.L, 256, 16);
    const bool bf = gd->feat_dtype == SNAKE_BF16;
#define SNAKE_HG_FWD(FF)                                                                              \
    if (bf)                                                                                           \
        hashgrid_fwd_kernel<FF, __hip_bfloat16><<<grid, 256, 0, st>>>(                                \
            g, table, pos, tile_id, sample_idx, n, n_dev, static_cast<__hip_bfloat16 *>(feat), idx_dbg); \
    else                                                                                              \
        hashgrid_fwd_kernel<FF, float><<<grid, 256, 0, st>>>(g, table, pos, tile_id, sample_idx, n,   \
                                                             n_dev, static_cast<float *>(feat), idx_dbg)
    if (F == 1) {
        SNAKE_HG_FWD(1);
    } else if (F == 2) {
        SNAKE_HG_FWD(2);
    } else {
        SNAKE_HG_FWD(4);
    }
#undef SNAKE_HG_FWD
    return launch_status(__func__);
}

int snake_hashgrid_bwd(const snake_grid_desc *gd, const float *pos, const uint8_t *tile_id,
                       const int32_t *sample_idx, int64_t n, const int64_t *n_dev, const float *dfeat,
                       float *dtable, snake_stream_t stream)
{
    Grid g;
    int rc = make_grid(gd, g, __func__);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_hashgrid_bwd: n < 0");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(pos);
    SNAKE_NOT_NULL(dfeat);
    SNAKE_NOT_NULL(dtable);
    const int F = gd->n_features;
    SNAKE_ALIGNED(dfeat, 4 * F);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned grid = grid_for(n * g.L, 256, 16);
    if (F == 1)
        hashgrid_bwd_kernel<1><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
    else if (F == 2)
        hashgrid_bwd_kernel<2><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
    else
        hashgrid_bwd_kernel<4><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
    return launch_status(__func__);
}

}  // extern "C"
