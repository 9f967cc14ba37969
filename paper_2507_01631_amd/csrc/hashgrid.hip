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

#include <type_traits>

#include "common.h"
#include "scan.h"

namespace snake {
namespace {

struct Grid {
    int K;                // tiles in the table
    unsigned int *err;    // device error word
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

// Identity of the cell holding x on a level of resolution N <= 256 in a
// tile: one byte per coordinate and the tile's index in the top byte.
__device__ __forceinline__ uint32_t cell_key(const Grid &g, int l, const float x[3], int64_t tile)
{
    const int N = g.res[l];
    uint32_t c[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cell(x[a], N, c[a], w[a]);
    return c[0] | (c[1] << 8) | (c[2] << 16) | ((uint32_t)tile << 24);
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

// Table entries: FP32, or the BF16 mirror of the forward (one 16-bit word
// per feature; widening to FP32 is a shift).  Pair loads fetch the slots
// (2m, 2m+1) of the x-neighbour pairing in one access.
template <int F, typename TabT>
struct Entry;
template <int F>
struct Entry<F, float> {
    typedef typename Vec<F>::T VT;
    __device__ static VT one(const float *lev, uint32_t i) { return reinterpret_cast<const VT *>(lev)[i]; }
};
__device__ __forceinline__ float bf16_bits(uint32_t h) { return __uint_as_float(h << 16); }
template <>
struct Entry<1, __hip_bfloat16> {
    __device__ static float one(const __hip_bfloat16 *lev, uint32_t i)
    {
        return bf16_bits(reinterpret_cast<const uint16_t *>(lev)[i]);
    }
};
template <>
struct Entry<2, __hip_bfloat16> {
    __device__ static float2 one(const __hip_bfloat16 *lev, uint32_t i)
    {
        const uint32_t w = reinterpret_cast<const uint32_t *>(lev)[i];
        return make_float2(bf16_bits(w & 0xffffu), bf16_bits(w >> 16));
    }
    // slots 2m and 2m+1 in one 8-byte load
    __device__ static void pair(const __hip_bfloat16 *lev, uint32_t m, float2 &lo, float2 &hi)
    {
        const uint2 w = reinterpret_cast<const uint2 *>(lev)[m];
        lo = make_float2(bf16_bits(w.x & 0xffffu), bf16_bits(w.x >> 16));
        hi = make_float2(bf16_bits(w.y & 0xffffu), bf16_bits(w.y >> 16));
    }
};
template <>
struct Entry<4, __hip_bfloat16> {
    __device__ static float4 one(const __hip_bfloat16 *lev, uint32_t i)
    {
        const uint2 w = reinterpret_cast<const uint2 *>(lev)[i];
        return make_float4(bf16_bits(w.x & 0xffffu), bf16_bits(w.x >> 16), bf16_bits(w.y & 0xffffu),
                           bf16_bits(w.y >> 16));
    }
};
template <>
struct Entry<2, float> {
    __device__ static float2 one(const float *lev, uint32_t i) { return reinterpret_cast<const float2 *>(lev)[i]; }
    __device__ static void pair(const float *lev, uint32_t m, float2 &lo, float2 &hi)
    {
        const float4 w = reinterpret_cast<const float4 *>(lev)[m];
        lo = make_float2(w.x, w.y);
        hi = make_float2(w.z, w.w);
    }
};

__device__ __forceinline__ void store_feat(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_feat(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }

// Four floats read with one 16-byte load from an 8-byte aligned address, and
// two words with one 8-byte load from a 4-byte aligned one.
typedef float F4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t U2a4 __attribute__((ext_vector_type(2), aligned(4)));

template <int F, typename OutT, typename TabT>
__global__ __launch_bounds__(256) void hashgrid_fwd_kernel(Grid g, const TabT *__restrict__ table,
                                                           const float *__restrict__ pos,
                                                           const uint8_t *__restrict__ tile_id,
                                                           const int32_t *__restrict__ sidx, int64_t n,
                                                           const int64_t *__restrict__ n_dev,
                                                           OutT *__restrict__ feat,
                                                           uint32_t *__restrict__ idx_dbg, int superchunk,
                                                           uint32_t levels)
{
    typedef typename Vec<F>::T VT;
    const int64_t ne = effective_n(n, n_dev);
    const int64_t chunks = (ne + 255) / 256;
    const int nl = __builtin_popcount(levels);      // the levels this launch gathers
    const int64_t units = chunks * nl;
    // super-chunks of sc chunks, every level of one before the next (sc =
    // chunks: level by level over all samples)
    const int64_t sc = superchunk > 0 && (int64_t)superchunk < chunks ? (int64_t)superchunk : chunks;
    const int64_t per = sc * nl;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t b = u / per, r = u - b * per;
        const int64_t c0 = b * sc;
        const int64_t se = chunks - c0 < sc ? chunks - c0 : sc;      // chunks of this super-chunk
        uint32_t lm = levels;
        for (int k = (int)(r / se); k > 0; --k) lm &= lm - 1;       // the k-th level of the set
        const int l = __builtin_ctz(lm);
        const int64_t rl = r / se;
        const int64_t s = (c0 + (r - rl * se)) * 256 + threadIdx.x;
        if (s >= ne) continue;
        const int64_t si = sidx ? sidx[s] : s;
        const float x[3] = {pos[3 * si], pos[3 * si + 1], pos[3 * si + 2]};
        const int64_t tile = tile_id ? tile_id[si] : 0;
        if (tile >= g.K) {                      // no such tile: zero features, flag it
            for (int f = 0; f < F; ++f) store_feat(feat + ((int64_t)l * n + s) * F + f, 0.0f);
            if (g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_TILE_ID);
            continue;
        }
        uint32_t idx[8];
        float wt[8];
        corners(g, l, x, idx, wt);
        const TabT *lev = table + ((tile * g.L + l) << g.log2T) * F;
        VT v[8];
        if constexpr (F == 2 && std::is_same<TabT, __hip_bfloat16>::value) {
            // BF16 entries are 4 bytes.  On a densely indexed level the
            // x-neighbours' slots are consecutive: one 8-byte load (4-byte
            // aligned) fetches both.  Elsewhere one 16-byte load covers an
            // aligned quad of slots, which holds both x-neighbours for three
            // pairs in four.
            const uint4 *lev4 = reinterpret_cast<const uint4 *>(lev);
            if ((g.dense_bits >> l) & 1u) {
                const uint32_t *lev1 = reinterpret_cast<const uint32_t *>(lev);
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const U2a4 w = *reinterpret_cast<const U2a4 *>(lev1 + idx[2 * p]);
                    v[2 * p] = make_float2(bf16_bits(w.x & 0xffffu), bf16_bits(w.x >> 16));
                    v[2 * p + 1] = make_float2(bf16_bits(w.y & 0xffffu), bf16_bits(w.y >> 16));
                }
            } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t a = idx[2 * p], b = idx[2 * p + 1];
                if ((a >> 2) == (b >> 2)) {
                    const uint4 w4 = lev4[a >> 2];
                    const uint32_t ka = a & 3u, kb = b & 3u;
                    const uint32_t wa = (ka & 2u) ? ((ka & 1u) ? w4.w : w4.z) : ((ka & 1u) ? w4.y : w4.x);
                    const uint32_t wb = (kb & 2u) ? ((kb & 1u) ? w4.w : w4.z) : ((kb & 1u) ? w4.y : w4.x);
                    v[2 * p] = make_float2(bf16_bits(wa & 0xffffu), bf16_bits(wa >> 16));
                    v[2 * p + 1] = make_float2(bf16_bits(wb & 0xffffu), bf16_bits(wb >> 16));
                } else {
                    v[2 * p] = Entry<F, TabT>::one(lev, a);
                    v[2 * p + 1] = Entry<F, TabT>::one(lev, b);
                }
            }
            }
        } else if constexpr (F == 2) {
            // corners q and q^1 differ only in x.  On a densely indexed level
            // their slots are always consecutive (a, a+1): one 16-byte load
            // (8-byte aligned) fetches both.  Elsewhere, when the slots are an
            // aligned pair (2m, 2m+1) -- half of all pairs -- one load fetches
            // both: one cache-line request, not two.
            if ((g.dense_bits >> l) & 1u) {
                const float *levf = reinterpret_cast<const float *>(lev);
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const F4a8 w = *reinterpret_cast<const F4a8 *>(levf + 2 * (size_t)idx[2 * p]);
                    v[2 * p] = make_float2(w.x, w.y);
                    v[2 * p + 1] = make_float2(w.z, w.w);
                }
            } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t a = idx[2 * p], b = idx[2 * p + 1];
                if ((a ^ b) == 1u) {
                    float2 lo, hi;
                    Entry<F, TabT>::pair(lev, a >> 1, lo, hi);
                    v[2 * p] = (a & 1u) ? hi : lo;
                    v[2 * p + 1] = (a & 1u) ? lo : hi;
                } else {
                    v[2 * p] = Entry<F, TabT>::one(lev, a);
                    v[2 * p + 1] = Entry<F, TabT>::one(lev, b);
                }
            }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = Entry<F, TabT>::one(lev, idx[q]);
        }
        float acc[F];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            acc[f] = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[f] = fmaf(wt[q], Vec<F>::get(v[q], f), acc[f]);
        }
        if constexpr (F == 2 && std::is_same<OutT, __hip_bfloat16>::value) {
            // both features of the sample-level in one 4-byte store
            const __hip_bfloat16 h0 = __float2bfloat16(acc[0]), h1 = __float2bfloat16(acc[1]);
            const uint32_t packed = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                                    ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
            *reinterpret_cast<uint32_t *>(feat + ((int64_t)l * n + s) * F) = packed;
        } else {
#pragma unroll
            for (int f = 0; f < F; ++f) store_feat(feat + ((int64_t)l * n + s) * F + f, acc[f]);
        }
        if (idx_dbg) {
#pragma unroll
            for (int q = 0; q < 8; ++q) idx_dbg[(s * g.L + l) * 8 + q] = idx[q];
        }
    }
}

// ---- forward from an LDS copy of the level slice ----------------------------
//
// Gathers through the vector memory path are served at about one cache line
// per clock per CU, so a wavefront's eight random corner loads per level cost
// hundreds of clocks even when the slice sits in L2.  A level whose slice of
// one tile (T entries, or (N+1)^3 on a densely indexed level) fits in LDS is
// therefore gathered from an LDS copy: a block takes kLdsR x kLdsThreads
// consecutive samples, keeps their positions in registers, and for each such
// level copies the slice of every tile its samples use into LDS with
// coalesced 16-byte loads, then reads the corners there.  Samples grouped by
// tile (as a window's partition leaves them) use one or two tiles per block;
// any order is correct, at one copy per tile between the block's smallest and
// largest tile id.  The corner arithmetic and the blend are those of the
// kernel above, so both give the same bits.
constexpr int kLdsThreads = 1024;
constexpr int kLdsR = 4;

template <int F, typename OutT>
__device__ __forceinline__ void store_feats(OutT *__restrict__ feat, int64_t at, const float (&acc)[F])
{
    if constexpr (F == 2 && std::is_same<OutT, __hip_bfloat16>::value) {
        const __hip_bfloat16 h0 = __float2bfloat16(acc[0]), h1 = __float2bfloat16(acc[1]);
        const uint32_t packed = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        *reinterpret_cast<uint32_t *>(feat + at * F) = packed;
    } else {
#pragma unroll
        for (int f = 0; f < F; ++f) store_feat(feat + at * F + f, acc[f]);
    }
}

// corners() with the indexing rule fixed at compile time (same arithmetic)
template <bool Dense>
__device__ __forceinline__ void corners_of(const Grid &g, int l, const float x[3], uint32_t idx[8], float wt[8])
{
    const int N = g.res[l];
    uint32_t c[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cell(x[a], N, c[a], w[a]);
    const uint32_t side = (uint32_t)N + 1u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t i = c[0] + (q & 1), j = c[1] + ((q >> 1) & 1), k = c[2] + ((q >> 2) & 1);
        idx[q] = Dense ? i + j * side + k * side * side
                       : ((i * 1u) ^ (j * 2654435761u) ^ (k * 805459861u)) & g.mask;
        const float wx = (q & 1) ? w[0] : 1.0f - w[0];
        const float wy = ((q >> 1) & 1) ? w[1] : 1.0f - w[1];
        const float wz = ((q >> 2) & 1) ? w[2] : 1.0f - w[2];
        wt[q] = (wx * wy) * wz;
    }
}

// One level of one tile for the block's samples of that tile, gathered from
// the slice copy in LDS.  s0 is the thread's first sample; its r-th sample
// is s0 + r * kLdsThreads.
template <bool Dense, int F, typename OutT, typename TabT>
__device__ __forceinline__ void lds_level(const Grid &g, int l, int t, const TabT *lev, const float (&x)[kLdsR][3],
                                          const int (&tl)[kLdsR], OutT *__restrict__ feat, int64_t n, int64_t s0,
                                          uint32_t *__restrict__ idx_dbg)
{
    typedef typename Vec<F>::T VT;
#pragma unroll
    for (int r = 0; r < kLdsR; ++r) {
        if (tl[r] != t) continue;
        const int64_t s = s0 + (int64_t)r * kLdsThreads;
        uint32_t idx[8];
        float wt[8];
        corners_of<Dense>(g, l, x[r], idx, wt);
        VT v[8];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            v[2 * p] = Entry<F, TabT>::one(lev, idx[2 * p]);
            // on a densely indexed level the x-neighbour holds the next slot
            v[2 * p + 1] = Entry<F, TabT>::one(lev, Dense ? idx[2 * p] + 1u : idx[2 * p + 1]);
        }
        float acc[F];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            acc[f] = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[f] = fmaf(wt[q], Vec<F>::get(v[q], f), acc[f]);
        }
        store_feats<F>(feat, (int64_t)l * n + s, acc);
        if (idx_dbg) {
#pragma unroll
            for (int q = 0; q < 8; ++q) idx_dbg[(s * g.L + l) * 8 + q] = idx[q];
        }
        // one sample at a time: interleaving them only adds registers
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int F, typename OutT, typename TabT>
__global__ __launch_bounds__(kLdsThreads) void hashgrid_fwd_lds_kernel(Grid g, const TabT *__restrict__ table,
                                                                      const float *__restrict__ pos,
                                                                      const uint8_t *__restrict__ tile_id,
                                                                      const int32_t *__restrict__ sidx, int64_t n,
                                                                      const int64_t *__restrict__ n_dev,
                                                                      OutT *__restrict__ feat,
                                                                      uint32_t *__restrict__ idx_dbg,
                                                                      uint32_t levels)
{
    extern __shared__ uint4 sslice[];
    __shared__ int srange[2];
    const TabT *lev = reinterpret_cast<const TabT *>(sslice);
    const int64_t ne = effective_n(n, n_dev);
    const int64_t per = (int64_t)kLdsThreads * kLdsR;
    const int64_t subs = (ne + per - 1) / per;
    const int tid = (int)threadIdx.x;
    for (int64_t b = blockIdx.x; b < subs; b += gridDim.x) {
        float x[kLdsR][3];
        int tl[kLdsR];
        int tmin = 0x7fffffff, tmax = -1;
#pragma unroll
        for (int r = 0; r < kLdsR; ++r) {
            const int64_t s = b * per + (int64_t)r * kLdsThreads + tid;
            tl[r] = -1;
            x[r][0] = x[r][1] = x[r][2] = 0.0f;
            if (s < ne) {
                const int64_t si = sidx ? sidx[s] : s;
                x[r][0] = pos[3 * si];
                x[r][1] = pos[3 * si + 1];
                x[r][2] = pos[3 * si + 2];
                const int t = tile_id ? (int)tile_id[si] : 0;
                if (t >= g.K) {                 // no such tile: zero features, flag it
                    const float z[F] = {};
                    for (uint32_t lm = levels; lm; lm &= lm - 1)
                        store_feats<F>(feat, (int64_t)__builtin_ctz(lm) * n + s, z);
                    if (g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_TILE_ID);
                } else {
                    tl[r] = t;
                    tmin = t < tmin ? t : tmin;
                    tmax = t > tmax ? t : tmax;
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int a = __shfl_xor(tmin, o, 64), c = __shfl_xor(tmax, o, 64);
            tmin = a < tmin ? a : tmin;
            tmax = c > tmax ? c : tmax;
        }
        __syncthreads();                        // the previous sub-range has read srange
        if (tid == 0) {
            srange[0] = 0x7fffffff;
            srange[1] = -1;
        }
        __syncthreads();
        if (lane_id() == 0) {
            atomicMin(&srange[0], tmin);
            atomicMax(&srange[1], tmax);
        }
        __syncthreads();
        const int t0 = srange[0], t1 = srange[1];
        for (uint32_t lm = levels; lm; lm &= lm - 1) {
            const int l = __builtin_ctz(lm);
            const bool dense = (g.dense_bits >> l) & 1u;
            const uint32_t side = (uint32_t)g.res[l] + 1u;
            const uint32_t entries = dense ? side * side * side : g.mask + 1u;
            const uint32_t nvec = (uint32_t)(((uint64_t)entries * F * sizeof(TabT) + 15) / 16);
            for (int t = t0; t <= t1; ++t) {
                __syncthreads();                // every gather from the previous copy is done
                const uint4 *src = reinterpret_cast<const uint4 *>(table + (((int64_t)t * g.L + l) << g.log2T) * F);
                // four 16-byte loads in flight per thread (a clamped index past
                // the end re-reads the last vector, which is not stored)
                for (uint32_t i0 = (uint32_t)tid; i0 < nvec; i0 += 4 * kLdsThreads) {
                    uint4 w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t i = i0 + (uint32_t)k * kLdsThreads;
                        w[k] = src[i < nvec ? i : nvec - 1];
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t i = i0 + (uint32_t)k * kLdsThreads;
                        if (i < nvec) sslice[i] = w[k];
                    }
                }
                __syncthreads();
                if (dense)
                    lds_level<true, F, OutT, TabT>(g, l, t, lev, x, tl, feat, n, b * per + tid, idx_dbg);
                else
                    lds_level<false, F, OutT, TabT>(g, l, t, lev, x, tl, feat, n, b * per + tid, idx_dbg);
            }
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
        if (tile >= g.K) {
            if (g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_TILE_ID);
            continue;
        }
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

// ---- binned adjoint ----------------------------------------------------------
//
// Global FP32 atomics on this chip run at a fixed ~2e10 operations/s whatever
// the footprint, far below the rate at which the samples produce corner
// gradients (L*8*F per sample).  The binned adjoint therefore sorts the
// corner contributions by table slot before adding them:
//   count   per (bin, block) how many (slot, w*g) items a block's samples
//           make, and each level's largest |dfeat|
//   scan    exclusive offsets, bin-major, so each bin's items are contiguous
//   scatter write the items to their bin (LDS cursors per block)
//   reduce  per equal share of the items: add into an LDS copy of the bin's
//           slots, then flush the bin once per touched slot into a pass-wide
//           integer accumulator of two 64-bit words (hi 2^52 + lo)
//   convert every accumulator slot of the pass, rounded once, into dtable
// A pass covers `lg` levels; bins never straddle levels.
//
// Item values.  Each stored value (one corner's w*g, or the FP32 sum of a run
// of consecutive samples of a ray in one cell) is rounded once to a 26-bit
// float: a sign, a 6-bit code exponent j and 19 stored mantissa bits.  With
// the level's top exponent Et = e + 7 (2^(e-1) <= max|dfeat of the level| <
// 2^e, so every value is below 2^(Et-1) even for a run of 64 lanes) a value
// |v| = 1.m * 2^(Et-k) has k = 1..63 and is stored with j = 64 - k (j = 0
// is the value 0), i.e. its biased FP32 exponent less a per-level base: the
// code is the rounded exponent-and-mantissa bits less a constant.  20
// significant bits (relative error at most 2^-20); values below 2^(Et-63) =
// 2^(e-56) are stored as zero.
//
// Exact sums.  LDS float atomics are slow on this chip (about 2e11/s) while
// LDS integer atomics are about 20x faster, so the values are summed as
// integers: a value with k <= 22 adds (2^19+m) << (22-k) into a "big"
// accumulator with unit 2^(Et-41); one with 22 < k <= 44 adds
// (2^19+m) << (44-k) into a "small" one with unit 2^(Et-63); smaller ones
// (k > 44, below 2^(e-37)) are rounded to that unit.  Each term is below 2^41
// and a block adds at most 2^21 items into one copy before flushing it, so
// the 64-bit LDS sums cannot overflow.  Integer sums do not depend on the
// order of addition, and the items do not depend on the grid (block ranges
// are whole 64-sample wavefronts), so the result is the same bits whatever
// the chunking, the scheduling or the grid.  The only roundings are the
// value's (2^-20 relative, or 2^(e-57) absolute below 2^(e-37)) and the
// final one to FP32, so every table entry keeps its own relative precision
// however small it is against the level's largest gradient.
//
// Consecutive samples of a ray that lie in one cell are first merged across
// the wavefront (whole runs, all eight corners at once), which shortens the
// item list on the coarse levels; an item is one 64-bit word for F <= 2.

constexpr int kBinBlocks = 2048;        // most count/scatter blocks (the workspace holds this many)
constexpr int kMaxBins = 4096;          // bins per pass (LDS counters)
constexpr int kAccWords = 8192;         // LDS accumulators: 2 x 8192 int64 = 128 KB
constexpr int kReduceThreads = 1024;    // reduce block: many loads in flight per CU
constexpr int kReducePerCU = 1;         // reduce blocks resident per CU (128 KB of LDS each)
constexpr int kRU = 6;                  // items in flight per thread in the reduce, per buffer (16
                                        // wavefronts per CU allow 128 registers; builds of this
                                        // kernel at exactly 128 have given wrong sums, so kRU keeps
                                        // it below that)
constexpr int64_t kFlushItems = 1 << 21;  // most items a block adds into its LDS copy between flushes

struct BinPlan {
    int l0, lg;            // levels [l0, l0 + lg) in this pass
    int kt2_log2;          // per-level key space (padded K*T), log2
    int binshift;          // slots per bin = 2^binshift
    int nbpl;              // bins per level
    int nb;                // bins in the pass
    int T_log2;
};

__device__ __forceinline__ bool wave_uniform(int b, bool active, int &b0)
{
    const unsigned long long act = __ballot(active);
    if (!act) return false;
    const int first = __ffsll((long long)act) - 1;
    b0 = __builtin_amdgcn_readlane(b, first);
    return __all(!active || b == b0);
}

template <int F>
__device__ __forceinline__ bool grad_nonzero(const typename Vec<F>::T &gv)
{
    bool any = false;
#pragma unroll
    for (int f = 0; f < F; ++f) any |= Vec<F>::get(gv, f) != 0.0f;
    return any;
}

// |x| as float bits (non-negative floats order as unsigned integers).
__device__ __forceinline__ uint32_t absbits(float x) { return __float_as_uint(x) & 0x7fffffffu; }
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

// Top exponent Et = e + 7 of a level's item values, from the bit pattern of
// its largest |dfeat| (2^(e-1) <= m < 2^e): a corner value w g (w <= 1) is
// below 2^e, a run of at most 64 of them below 2^(e+6) = 2^(Et-1).
__device__ __forceinline__ int level_top(uint32_t maxbits)
{
    if (maxbits == 0u || maxbits >= 0x7f800000u) return 0;
    int e;
    frexpf(__uint_as_float(maxbits), &e);
    return e + 7;
}

// A level takes part when it has a nonzero, finite largest gradient.
__device__ __forceinline__ bool level_ok(uint32_t maxbits) { return maxbits != 0u && maxbits < 0x7f800000u; }

// Consecutive lanes (consecutive samples of a ray) often hit the same slot on
// coarse levels.  Each run of equal keys across the wavefront emits one item,
// from its last lane, holding the run's sum.  run_bounds gives this lane's
// run start rs, whether it emits (rtail), and the wave's active lanes and run
// heads; when no run is longer than one lane it reports exactly that
// (heads == acts) without the rest.
__device__ __forceinline__ void run_bounds(uint32_t key, bool act, unsigned long long &acts,
                                           unsigned long long &heads, int &rs, bool &rtail)
{
    const int lane = lane_id();
    const uint32_t pk = __shfl_up(key, 1, 64);
    const bool pa = __shfl_up(act ? 1 : 0, 1, 64) != 0;
    const bool head = act && (lane == 0 || !pa || pk != key);
    heads = __ballot(head);
    acts = __ballot(act);
    if (heads == acts) {
        rs = lane;
        rtail = act;
        return;
    }
    const uint32_t nk = __shfl_down(key, 1, 64);
    const bool na = __shfl_down(act ? 1 : 0, 1, 64) != 0;
    rtail = act && (lane == 63 || !na || nk != key);
    // start of this lane's run: highest head at or below this lane
    const unsigned long long le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const unsigned long long hb = heads & le;
    rs = hb ? 63 - __clzll((long long)hb) : lane;
}

// Sum each run across the wavefront (segmented inclusive scan, FP32) for all
// eight corners at once: a run is a stretch of consecutive active lanes whose
// samples lie in one cell (cellkey), so every corner of the cell has the same
// key along it.  Returns whether this lane emits the run's eight items, with
// v the run totals there.  The additions follow the lanes' positions in the
// wavefront only, and wavefronts always cover the same 64 samples, so the
// sums are the same bits for any grid.
template <int F>
__device__ __forceinline__ bool merge_runs(uint32_t cellkey, bool act, float (&v)[8][F])
{
    const int lane = lane_id();
    unsigned long long acts, heads;
    int rs;
    bool rtail;
    run_bounds(cellkey, act, acts, heads, rs, rtail);
    if (heads == acts) return act;                 // no run longer than one lane
    // Scan steps d = 1, 2, ... complete every run of up to 2d lanes; c holds
    // the lanes that end d consecutive continuation lanes (active lanes that
    // are not a run's head) and is zero once no run exceeds the steps taken.
    // The count is the same on every lane (it comes from ballots).
    unsigned long long c = acts & ~heads;
    for (int d = 1; d < 64 && c != 0ull; d <<= 1) {
        const bool take = lane - d >= rs;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const float u = __shfl_up(v[q][f], d, 64);
                if (take) v[q][f] += u;
            }
        }
        c &= c >> d;
    }
    return rtail;
}

// The lane that emits a run's items; the same decision as merge_runs, without
// the sums (the count pass needs only how many items).
__device__ __forceinline__ bool run_tail(uint32_t cellkey, bool act)
{
    unsigned long long acts, heads;
    int rs;
    bool rtail;
    run_bounds(cellkey, act, acts, heads, rs, rtail);
    return rtail;
}

// A level's item code: the biased exponent B - 1 that code exponent 0 sits
// below (B = Et + 64, at least 1, so that code exponent j = 1 holds
// 2^(Et-63) whenever Et + 64 >= 1), and k0 with k = k0 - j, the distance of
// a value's exponent below Et (1..63 for every value of the level).
struct LevelCode {
    uint32_t base;      // (B - 1) << 19
    int k0;             // Et + 128 - B
};
__device__ __forceinline__ LevelCode level_code(int Et)
{
    const int B = Et + 64 > 1 ? Et + 64 : 1;
    return LevelCode{(uint32_t)(B - 1) << 19, Et + 128 - B};
}

// 26-bit item value of v (see above): sign in bit 25, code exponent j (1..63;
// 0 only for the value 0) in bits 19..24, mantissa rounded to 19 bits
// (nearest, ties to even) in bits 0..18.  The rounded exponent and mantissa
// less the level's base are j and the mantissa at once (a carry out of the
// mantissa moves into the exponent, as it should).  Zeros, subnormals and
// values below the level's range are stored as 0.
__device__ __forceinline__ uint32_t val_encode(float v, uint32_t base)
{
    const uint32_t u = __float_as_uint(v);
    const uint32_t a = u & 0x7fffffffu;
    const uint32_t r = (a + 0x7u + ((a >> 4) & 1u)) >> 4;
    const uint32_t d = r - base;
    // every value is below 2^(Et-1), so j <= 63 unless v is not finite (a
    // level with a non-finite gradient stores zeros before this point)
    return d - (1u << 19) < (63u << 19) ? (d | ((u >> 6) & (1u << 25))) : 0u;
}

// An item is one 64-bit word (F = 1, 2) or two (F = 4): the F 26-bit values
// from bit 0 up (the fourth feature's pair in the second word), and the slot
// within the bin in the top bits of the first word (from bit 26 for F = 1,
// bit 52 otherwise: at most 13 and 12 bits).
constexpr int kValBits = 26;
constexpr uint32_t kValMask = (1u << kValBits) - 1u;

template <int F>
struct ItemFmt {
    static constexpr int NW = F == 4 ? 2 : 1;
};

template <int F>
__device__ __forceinline__ void item_pack(unsigned long long *dst, uint32_t slot, const uint32_t *v)
{
    if constexpr (F == 1) {
        dst[0] = (unsigned long long)v[0] | ((unsigned long long)slot << kValBits);
    } else {
        const uint32_t lo = v[0] | (v[1] << kValBits);
        const uint32_t hi = (v[1] >> (32 - kValBits)) | (slot << 20);
        dst[0] = (unsigned long long)lo | ((unsigned long long)hi << 32);
    }
    if constexpr (F == 4) dst[1] = (unsigned long long)v[2] | ((unsigned long long)v[3] << kValBits);
}

template <int F>
__device__ __forceinline__ void item_unpack(const unsigned long long *src, uint32_t &slot, uint32_t (&v)[F])
{
    const uint64_t w0 = src[0];
    const uint32_t lo = (uint32_t)w0, hi = (uint32_t)(w0 >> 32);
    if constexpr (F == 1) {
        slot = (uint32_t)(w0 >> kValBits);
        v[0] = lo & kValMask;
    } else {
        slot = hi >> 20;
        v[0] = lo & kValMask;
        v[1] = ((lo >> kValBits) | (hi << (32 - kValBits))) & kValMask;
    }
    if constexpr (F == 4) {
        const uint64_t w1 = src[1];
        v[2] = (uint32_t)w1 & kValMask;
        v[3] = (uint32_t)(w1 >> kValBits) & kValMask;
    }
}

// Adds a 26-bit value into the big (unit 2^(Et-41)) or the small (unit
// 2^(Et-63)) LDS accumulator, without branches (a zero value adds 0).
__device__ __forceinline__ void val_accumulate(uint32_t code, int k0, unsigned long long *big,
                                               unsigned long long *small)
{
    const int k = k0 - (int)((code >> 19) & 63u);       // k0 for the value 0
    const uint32_t m = code ? ((code & 0x7ffffu) | 0x80000u) : 0u;
    const bool isbig = k <= 22;
    const int sh = (isbig ? 22 : 44) - k;        // -19 .. 21 for the values (k = 1..63)
    // the signed value +-m 2^sh in the unit, below 2^(Et-44) (sh < 0) rounded
    // to it, halves away from 0: x = +-m 2^(sh+21) is exact in 64 bits, and
    // (x + 2^20 - [x < 0]) >> 21, shifting arithmetically, is that rounding
    const int32_t s = (int32_t)(code << 6) >> 31;                      // -1 when negative
    const int32_t ms = (int32_t)((m ^ (uint32_t)s) - (uint32_t)s);
    const int64_t x = (int64_t)((uint64_t)(int64_t)ms << (sh + 21));
    atomicAdd(isbig ? big : small, (unsigned long long)((x + ((int64_t)1 << 20) + s) >> 21));
}

// Samples of this count/scatter block: a contiguous range of whole 64-sample
// wavefronts, so that every wavefront covers the same samples (and merges the
// same runs) whatever the grid.
__device__ __forceinline__ void block_range(int64_t ne, int64_t &s0, int64_t &s1)
{
    const int64_t nw = (ne + 63) >> 6;
    s0 = (nw * blockIdx.x / gridDim.x) << 6;
    s1 = (nw * (blockIdx.x + 1) / gridDim.x) << 6;
    s0 = s0 < ne ? s0 : ne;
    s1 = s1 < ne ? s1 : ne;
}

// Runs of equal slots along a ray are worth merging only where cells are
// large against the sample spacing; on finer levels every item is emitted.
constexpr int kMergeMaxRes = 256;

template <int F>
__global__ __launch_bounds__(256) void bin_count_kernel(Grid g, BinPlan bp, const float *__restrict__ pos,
                                                        const uint8_t *__restrict__ tile_id,
                                                        const int32_t *__restrict__ sidx, int64_t n,
                                                        const int64_t *__restrict__ n_dev,
                                                        const float *__restrict__ dfeat,
                                                        uint32_t *__restrict__ lmax,
                                                        int32_t *__restrict__ counts)
{
    typedef typename Vec<F>::T VT;
    __shared__ int hist[kMaxBins];
    __shared__ uint32_t hmax[SNAKE_MAX_LEVELS];
    for (int b = threadIdx.x; b < bp.nb; b += blockDim.x) hist[b] = 0;
    if (threadIdx.x < SNAKE_MAX_LEVELS) hmax[threadIdx.x] = 0u;
    __syncthreads();
    int64_t s0, s1;
    block_range(effective_n(n, n_dev), s0, s1);
    const int lane = lane_id();
    for (int64_t base = s0; base < s1; base += blockDim.x) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < s1;
        float x[3] = {0.f, 0.f, 0.f};
        int64_t tile = 0;
        if (valid) {
            const int64_t si = sidx ? sidx[s] : s;
            x[0] = pos[3 * si];
            x[1] = pos[3 * si + 1];
            x[2] = pos[3 * si + 2];
            tile = tile_id ? tile_id[si] : 0;
        }
        const bool tile_ok = tile < g.K;
        if (valid && !tile_ok && g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_TILE_ID);
        const bool live = valid && tile_ok;
        // the level's gradients, loaded one level ahead; lanes past the range
        // read the block's first sample (a valid address) and discard it
        const int64_t sl = valid ? s : s0;
        VT gnext = *reinterpret_cast<const VT *>(dfeat + ((int64_t)bp.l0 * n + sl) * F);
        for (int lr = 0; lr < bp.lg; ++lr) {
            const int l = bp.l0 + lr;
            const bool dense_l = (g.dense_bits >> l) & 1u;
            const bool merge_l = g.res[l] <= kMergeMaxRes;
            const VT gv = gnext;
            if (lr + 1 < bp.lg) gnext = *reinterpret_cast<const VT *>(dfeat + ((int64_t)(l + 1) * n + sl) * F);
            // whether the sample contributes does not depend on its level's
            // largest |dfeat| (the scatter emits the same items, with zero
            // values for a level that holds a non-finite value); that maximum
            // is taken here, for the scatter's fixed-point scale
            const bool act = live && grad_nonzero<F>(gv);
            uint32_t gm = 0u;
            if (live) {
#pragma unroll
                for (int f = 0; f < F; ++f) gm = umax(gm, absbits(Vec<F>::get(gv, f)));
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) gm = umax(gm, (uint32_t)__shfl_xor((int)gm, d, 64));
            if (lane == 0 && gm) atomicMax(&hmax[lr], gm);
            uint32_t idx[8];
            float wt[8];
            corners(g, l, x, idx, wt);
            if (!merge_l && !dense_l) {
                // every corner of an active lane emits: one branch for all eight
                if (act) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        atomicAdd(&hist[lr * bp.nbpl + (int)((((uint32_t)tile << bp.T_log2) + idx[q]) >> bp.binshift)],
                                  1);
                }
                continue;
            }
            // on merged levels a run of samples in one cell emits one item per
            // corner, from its last lane
            const bool emit = merge_l ? run_tail(cell_key(g, l, x, tile), act) : act;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t key = ((uint32_t)tile << bp.T_log2) + idx[q];
                const int b = lr * bp.nbpl + (int)(key >> bp.binshift);
                int b0;
                // the vote must run on every lane: inside the leader's branch
                // EXEC holds one lane and the popcount would be 1
                const unsigned long long am = __ballot(emit);
                // a whole wavefront lands in one bin only on the coarse, densely
                // indexed levels; elsewhere the vote would cost more than it saves
                if (dense_l && wave_uniform(b, emit, b0)) {
                    if (lane == __ffsll((long long)am) - 1) atomicAdd(&hist[b0], __popcll(am));
                } else if (emit) {
                    atomicAdd(&hist[b], 1);
                }
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bp.nb; b += blockDim.x) counts[(int64_t)b * gridDim.x + blockIdx.x] = hist[b];
    if (threadIdx.x < bp.lg && hmax[threadIdx.x]) {
        const uint32_t m = hmax[threadIdx.x];
        if (m >= 0x7f800000u && g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_NONFINITE);
        atomicMax(&lmax[bp.l0 + threadIdx.x], m);
    }
}

// Scatter block: 512 threads (a batch of 4096 items) for one-word items,
// 256 for two-word ones (F = 4), so the staging stays within 64 KB of LDS.
// For one-word items the kernel is held to 80 registers, so three blocks
// (24 wavefronts) share a CU: the batches' barriers leave fewer idle cycles.
template <int F>
struct ScatterShape {
    static constexpr int threads = F == 4 ? 256 : 512;
    static constexpr int batch = threads * 8;      // items of one (chunk, level) batch at most
    static constexpr int waves_per_simd = F == 4 ? 1 : 6;
};
constexpr size_t kScatterLds = 64 * 1024;
constexpr int kDropped = INT32_MIN;                 // a bin whose batch is not written

// Dynamic LDS of the scatter pass, in bytes: the staged items (8-byte words,
// first, for alignment), their bins (16-bit), then the int arrays.
static size_t scatter_lds_bytes(int nb, int nbpl, int F)
{
    const size_t nw = F == 4 ? 2 : 1;
    const size_t threads = F == 4 ? ScatterShape<4>::threads : ScatterShape<1>::threads;
    return threads * 8 * (8 * nw + 2) + sizeof(int) * ((size_t)2 * nb + (size_t)3 * nbpl + 1);
}

// Each (chunk, level) batch of items is encoded in registers, counting-sorted
// by bin into LDS, then written out in that order, so consecutive lanes store
// consecutive item slots of one bin instead of each lane hitting its own
// random cache line.  The next level's gradients are loaded while the
// current level is sorted.
template <int F>
__global__ __launch_bounds__(ScatterShape<F>::threads) __attribute__((amdgpu_waves_per_eu(ScatterShape<F>::waves_per_simd))) void bin_scatter_kernel(Grid g, BinPlan bp, const float *__restrict__ pos,
                                                                      const uint8_t *__restrict__ tile_id,
                                                                      const int32_t *__restrict__ sidx, int64_t n,
                                                                      const int64_t *__restrict__ n_dev,
                                                                      const float *__restrict__ dfeat,
                                                                      const int32_t *__restrict__ offsets,
                                                                      const int32_t *__restrict__ counts,
                                                                      const uint32_t *__restrict__ lmax,
                                                                      unsigned long long *__restrict__ items,
                                                                      int64_t dummy)
{
    typedef typename Vec<F>::T VT;
    constexpr int NW = ItemFmt<F>::NW;
    constexpr int NT = ScatterShape<F>::threads;
    constexpr int kScatterBatch = ScatterShape<F>::batch;
    extern __shared__ unsigned long long sm64[];
    unsigned long long *sitem = sm64;                                         // [batch][NW], bin-sorted
    uint16_t *sbin = reinterpret_cast<uint16_t *>(sitem + kScatterBatch * NW);  // [batch] bin in the level
    int *cursor = reinterpret_cast<int *>(sbin + kScatterBatch);             // [nb] next free item of the range
    int *cend = cursor + bp.nb;                                              // [nb] end of this block's range
    int *hcnt = cend + bp.nb;                                                // [nbpl] items of the batch per bin
    int *hoff = hcnt + bp.nbpl;                                              // [nbpl] their start in the staging
    int *delta = hoff + bp.nbpl;                                             // [nbpl] global - staging index
    int *wtot = delta + bp.nbpl;                                             // [1] the batch's item count
    for (int b = threadIdx.x; b < bp.nb; b += blockDim.x) {
        const int64_t i = (int64_t)b * gridDim.x + blockIdx.x;
        cursor[b] = offsets[i];
        cend[b] = offsets[i] + counts[i];
    }
    for (int b = threadIdx.x; b < bp.nbpl; b += blockDim.x) hcnt[b] = 0;
    __syncthreads();
    int64_t s0, s1;
    block_range(effective_n(n, n_dev), s0, s1);
    const int lane = lane_id();
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t smask = (1u << bp.binshift) - 1u;
    for (int64_t base = s0; base < s1; base += NT) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < s1;
        // lanes past the range read the block's first sample (a valid
        // address) and discard it; the loads are branch-free
        const int64_t sl = valid ? s : s0;
        const int64_t si = sidx ? sidx[sl] : sl;
        const float x[3] = {pos[3 * si], pos[3 * si + 1], pos[3 * si + 2]};
        const int64_t tile = tile_id ? tile_id[si] : 0;
        const bool live = valid && tile < g.K;
        VT gnext = *reinterpret_cast<const VT *>(dfeat + ((int64_t)bp.l0 * n + sl) * F);
        for (int lr = 0; lr < bp.lg; ++lr) {
            const int l = bp.l0 + lr;
            const bool dense_l = (g.dense_bits >> l) & 1u;
            const bool merge_l = g.res[l] <= kMergeMaxRes;
            const uint32_t lm = lmax[l];
            const uint32_t cbase = level_code(level_top(lm)).base;
            const bool lok = level_ok(lm);
            VT gv = gnext;
            if (lr + 1 < bp.lg) gnext = *reinterpret_cast<const VT *>(dfeat + ((int64_t)(l + 1) * n + sl) * F);
            // the same decision as the count pass; a level without a finite,
            // nonzero maximum emits its items with zero values
            const bool act = live && grad_nonzero<F>(gv);
            if (!live || !lok) gv = VT{};
            uint32_t idx[8];
            float wt[8];
            corners(g, l, x, idx, wt);
            // 1. rank every emitted item within its bin for this batch
            uint32_t key[8];
            int rank[8];
            float v[8][F];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                key[q] = ((uint32_t)tile << bp.T_log2) + idx[q];
#pragma unroll
                for (int f = 0; f < F; ++f) v[q][f] = wt[q] * Vec<F>::get(gv, f);
                rank[q] = -1;
            }
            if (!merge_l && !dense_l) {
                // every corner of an active lane emits: one branch for all eight
                if (act) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) rank[q] = atomicAdd(&hcnt[key[q] >> bp.binshift], 1);
                }
            } else {
                const bool emit = merge_l ? merge_runs<F>(cell_key(g, l, x, tile), act, v) : act;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int bl = (int)(key[q] >> bp.binshift);
                    int b0;
                    if (dense_l && wave_uniform(bl, emit, b0)) {
                        const unsigned long long am = __ballot(emit);
                        const int leader = __ffsll((long long)am) - 1;
                        int r0 = 0;
                        if (lane == leader) r0 = atomicAdd(&hcnt[b0], __popcll(am));
                        r0 = __builtin_amdgcn_readlane(r0, leader);
                        rank[q] = emit ? r0 + __popcll(am & lt_mask) : -1;
                    } else if (emit) {
                        rank[q] = atomicAdd(&hcnt[bl], 1);
                    }
                }
            }
            // (this barrier also ends the previous batch's write-out on every
            // wavefront, so its staging and offsets may be overwritten below)
            __syncthreads();
            // 3. one wavefront: staging offsets (exclusive scan of the bin
            // counts), this block's global slots for each bin, counts reset
            if (threadIdx.x < 64) {
                const int per = (bp.nbpl + 63) >> 6;
                const int b0 = lane * per;
                int sum = 0;
                for (int k = 0; k < per; ++k)
                    if (b0 + k < bp.nbpl) sum += hcnt[b0 + k];
                int inc = sum;
#pragma unroll
                for (int dd = 1; dd < 64; dd <<= 1) {
                    const int u = __shfl_up(inc, dd, 64);
                    if (lane >= dd) inc += u;
                }
                int run = inc - sum;
                for (int k = 0; k < per; ++k) {
                    const int bl = b0 + k;
                    if (bl >= bp.nbpl) break;
                    const int c = hcnt[bl];
                    hcnt[bl] = 0;
                    hoff[bl] = run;
                    if (c > 0) {
                        const int b = lr * bp.nbpl + bl;
                        const int at = cursor[b];
                        cursor[b] = at + c;
                        if (at + c > cend[b]) {        // count and scatter disagree: never write past the range
                            if (g.err) atomicOr(g.err, (unsigned)SNAKE_DEVERR_INTERNAL);
                            delta[bl] = kDropped;
                        } else {
                            delta[bl] = at - run;
                        }
                    }
                    run += c;
                }
                if (lane == 63) wtot[0] = inc;
            }
            __syncthreads();
            const int total = wtot[0];
            // 4. counting-sort the batch into the staging area, in the items'
            // stored form (the level's scale is known)
            auto stage_item = [&](int q) {
                const int bl = (int)(key[q] >> bp.binshift);
                const int at = hoff[bl] + rank[q];
                uint32_t code[F];
#pragma unroll
                for (int f = 0; f < F; ++f) code[f] = val_encode(v[q][f], cbase);
                item_pack<F>(sitem + at * NW, key[q] & smask, code);
                sbin[at] = (uint16_t)bl;
            };
            if (!merge_l && !dense_l) {
                if (act) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) stage_item(q);
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (rank[q] >= 0) stage_item(q);
            }
            __syncthreads();
            // 5. write out: consecutive threads, consecutive slots of a bin.
            // Branch-free: a lane with no item (past the batch, or in a bin
            // the count did not allow) writes the dummy item, so every lane
            // issues the same stores and the next level's gradient load can
            // be waited for without draining them.
            {
                constexpr int U = kScatterBatch / NT;
                int jj[U], d[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = threadIdx.x + u * NT;
                    jj[u] = j < total ? j : -1;
                    d[u] = sbin[j];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) d[u] = delta[jj[u] >= 0 ? d[u] : 0];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = threadIdx.x + u * NT;
                    const int64_t dst = (jj[u] >= 0 && d[u] != kDropped) ? (int64_t)(j + d[u]) : dummy;
#pragma unroll
                    for (int k = 0; k < NW; ++k) items[dst * NW + k] = sitem[j * NW + k];
                }
            }
        }
    }
}



// dst = src rounded to BF16 (nearest, ties to even; NaN stays NaN).
__global__ __launch_bounds__(256) void to_bf16_kernel(const float4 *__restrict__ src, int64_t n4,
                                                      uint2 *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = src[i];
        const float f[4] = {v.x, v.y, v.z, v.w};
        uint32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t u = __float_as_uint(f[k]);
            h[k] = (u & 0x7fffffffu) > 0x7f800000u ? ((u >> 16) | 0x40u)
                                                   : ((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        }
        dst[i] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
}

__global__ void zero_u32_kernel(uint32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Largest bin b (in [0, nb)) whose first item index offsets[b nblk] is at
// most i: the bin holding item i (empty bins before it share its start).
__device__ __forceinline__ int bin_of_item(const int32_t *offsets, int nblk, int nb, int64_t i)
{
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)offsets[(int64_t)mid * nblk] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int F>
__global__ __launch_bounds__(kReduceThreads) void bin_reduce_kernel(BinPlan bp, const int32_t *__restrict__ offsets,
                                                                    int nblk, const int64_t *__restrict__ n_items,
                                                                    const unsigned long long *__restrict__ items,
                                                                    const uint32_t *__restrict__ lmax,
                                                                    unsigned long long *__restrict__ acc)
{
    // the bin's slots, feature-major (random slots spread over twice the
    // banks): big[f * slots + slot] and small[...] (units 2^(Et-41), 2^(Et-63))
    __shared__ unsigned long long big[kAccWords];
    __shared__ unsigned long long small[kAccWords];
    const int64_t total = *n_items;
    const int slots = 1 << bp.binshift;
    constexpr int NW = ItemFmt<F>::NW;
    // one contiguous, equal share of the pass's items per block (the grid is
    // what the chip holds at once, so there is no tail of late blocks)
    const int64_t c0 = total * blockIdx.x / gridDim.x, c1 = total * (blockIdx.x + 1) / gridDim.x;
    if (c0 >= c1) return;
    // the bins holding the share's first and last items (items carry only
    // their slot within the bin)
    const int bfirst = bin_of_item(offsets, nblk, bp.nb, c0);
    const int blast = bin_of_item(offsets, nblk, bp.nb, c1 - 1);
    for (int b = bfirst; b <= blast; ++b) {
        const int64_t bs = offsets[(int64_t)b * nblk];
        const int64_t be = b + 1 < bp.nb ? (int64_t)offsets[(int64_t)(b + 1) * nblk] : total;
        const int64_t blo = bs > c0 ? bs : c0, bhi = be < c1 ? be : c1;
        if (blo >= bhi) continue;
        // the bin's first key: level and table position of slot 0
        const uint32_t kbase = (uint32_t)b << bp.binshift;
        const int lr = (int)(kbase >> bp.kt2_log2);
        if (!level_ok(lmax[bp.l0 + lr])) continue;          // block-uniform
        const int k0 = level_code(level_top(lmax[bp.l0 + lr])).k0;
        unsigned long long *dst = acc + (((int64_t)lr << bp.kt2_log2) + (int64_t)(kbase & ((1u << bp.kt2_log2) - 1u))) * F * 2;
        // at most kFlushItems items between flushes keep the LDS sums in range
        for (int64_t lo = blo; lo < bhi; lo += kFlushItems) {
            const int64_t hi = lo + kFlushItems < bhi ? lo + kFlushItems : bhi;
            for (int e = threadIdx.x; e < slots * F; e += blockDim.x) {
                big[e] = 0ull;
                small[e] = 0ull;
            }
            __syncthreads();
            // kRU items per thread per round, and the next round's loads issued
            // before this round's additions, keep enough loads in flight.  The
            // loads are branch-free: past the end they re-read the last item,
            // which then adds zero.
            const int64_t stride = (int64_t)kRU * blockDim.x;
            unsigned long long wa[kRU][NW], wb[kRU][NW];
            auto load = [&](unsigned long long (&w)[kRU][NW], int64_t i0) {
#pragma unroll
                for (int u = 0; u < kRU; ++u) {
                    int64_t i = i0 + (int64_t)u * blockDim.x;
                    i = i < hi ? i : hi - 1;
#pragma unroll
                    for (int k = 0; k < NW; ++k) w[u][k] = items[i * NW + k];
                }
            };
            auto add = [&](const unsigned long long (&w)[kRU][NW], int64_t i0) {
#pragma unroll
                for (int u = 0; u < kRU; ++u) {
                    const bool ok = i0 + (int64_t)u * blockDim.x < hi;
                    uint32_t slot;
                    uint32_t v[F];
                    item_unpack<F>(w[u], slot, v);
#pragma unroll
                    for (int f = 0; f < F; ++f)
                        val_accumulate(ok ? v[f] : 0u, k0, &big[f * slots + slot], &small[f * slots + slot]);
                }
            };
            // the rounds alternate between the two buffers (unrolled by two);
            // every load is unconditional, so the compiler can count them
            // (the scheduling barriers keep the compiler from sinking a round's
            // loads below the previous round's additions)
            int64_t i0 = lo + threadIdx.x;
            load(wa, i0);
            while (i0 < hi) {
                load(wb, i0 + stride);
                __builtin_amdgcn_sched_barrier(0);
                add(wa, i0);
                i0 += stride;
                if (i0 >= hi) break;
                load(wa, i0 + stride);
                __builtin_amdgcn_sched_barrier(0);
                add(wb, i0);
                i0 += stride;
            }
            __syncthreads();
            // W = big 2^22 + small (in units of 2^(Et-63)) as hi 2^52 + lo with
            // |lo| < 2^51, added with 64-bit integer atomics into the pass-wide
            // accumulator (exact, so the order of the flushes is irrelevant; a
            // slot takes at most a few thousand flushes, so lo cannot overflow);
            // hi is zero, and skipped, unless |W| >= 2^51
            for (int e = threadIdx.x; e < slots * F; e += blockDim.x) {
                const int sl = e / F, f = e - sl * F;
                const long long A = (long long)big[f * slots + sl], B = (long long)small[f * slots + sl];
                if ((A | B) == 0) continue;
                const long long s0 = ((A & ((1ll << 30) - 1)) << 22) + (B & ((1ll << 52) - 1));   // [0, 2^53)
                const long long h0 = (A >> 30) + (B >> 52);
                const long long q = (s0 + (1ll << 51)) >> 52;                                       // 0, 1 or 2
                const long long wlo = s0 - (q << 52), whi = h0 + q;
                if (wlo) atomicAdd(dst + 2 * e, (unsigned long long)wlo);
                if (whi) atomicAdd(dst + 2 * e + 1, (unsigned long long)whi);
            }
            __syncthreads();
        }
    }
}

// x 2^p as FP32 for x = (hi 2^64 + lo), given as sign and magnitude, rounded
// once to nearest (ties to even) with integer operations only.  (A result
// below FP32's normal range is rounded a second time by the scaling.)
__device__ __forceinline__ float scaled_u128(bool neg, uint64_t hi, uint64_t lo, int p)
{
    float r;
    if (hi == 0 && lo < (1ull << 24)) {
        r = ldexpf((float)(uint32_t)lo, p);      // the integer is exact in FP32
    } else {
        const int bl = hi ? 128 - __clzll((long long)hi) : 64 - __clzll((long long)lo);   // bit length, > 24
        const int sh = bl - 24;                  // >= 1
        // the top 24 bits, the bit below them, and whether anything below that is set
        uint64_t top, half, sticky;
        if (sh >= 64) {
            const int rb = sh - 64;              // bits of hi below the top 24
            top = hi >> rb;
            if (rb == 0) {
                half = lo >> 63;
                sticky = lo & ~(1ull << 63);
            } else {
                const uint64_t below = hi & ((1ull << rb) - 1ull);
                half = (below >> (rb - 1)) & 1ull;
                sticky = (below & ((1ull << (rb - 1)) - 1ull)) | lo;
            }
        } else {
            top = (lo >> sh) | (hi << (64 - sh));   // x < 2^(sh+24): the shifted value has 24 bits
            half = (lo >> (sh - 1)) & 1ull;
            sticky = lo & ((1ull << (sh - 1)) - 1ull);
        }
        if (half && (sticky || (top & 1ull))) ++top;     // 2^24 stays exact
        r = ldexpf((float)(uint32_t)top, sh + p);
    }
    return neg ? -r : r;
}

// dtable += the pass's exact sums, hi 2^52 + lo units of 2^(Et-63), rounded
// once to FP32 (one value per table entry).
template <int F>
__global__ __launch_bounds__(256) void bin_convert_kernel(BinPlan bp, int L, const unsigned long long *__restrict__ acc,
                                                          const uint32_t *__restrict__ lmax, int K,
                                                          float *__restrict__ dtable)
{
    const int64_t per_level = ((int64_t)K << bp.T_log2) * F;    // real (unpadded) keys
    const int64_t total = per_level * bp.lg;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int lr = (int)(e / per_level);
        const int64_t r = e - (int64_t)lr * per_level;              // key * F + f
        const int64_t a = (((int64_t)lr << bp.kt2_log2) * F + r) * 2;
        const long long lo = (long long)acc[a], hi = (long long)acc[a + 1];
        if ((lo | hi) == 0) continue;
        // V = hi 2^52 + lo as a 128-bit two's-complement pair (vh, vl)
        uint64_t vl = (uint64_t)lo + ((uint64_t)hi << 52);
        const uint64_t carry = vl < (uint64_t)lo ? 1ull : 0ull;
        uint64_t vh = (uint64_t)((hi >> 12) + (lo >> 63)) + carry;
        const bool neg = (int64_t)vh < 0;
        if (neg) {                               // magnitude
            vl = ~vl + 1ull;
            vh = ~vh + (vl == 0ull ? 1ull : 0ull);
        }
        const int64_t key = r / F, f = r - key * F;
        const int64_t tile = key >> bp.T_log2, idx = key & ((1ll << bp.T_log2) - 1);
        const int Et = level_top(lmax[bp.l0 + lr]);
        dtable[((tile * L + bp.l0 + lr) << bp.T_log2) * F + idx * F + f] += scaled_u128(neg, vh, vl, Et - 63);
    }
}

struct BinWs {
    int32_t *counts, *offsets;
    int64_t *bsum, *n_items;
    uint32_t *lmax;
    unsigned long long *acc64;
    unsigned long long *items;
    int64_t item_cap;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of a pass over lg levels for n samples: counts, offsets, scan
// sums, the item count, per-level maxima, the pass's integer accumulator
// (lg x 2^kt2 x F x two int64) and the items (with one dummy item past the
// last, which the scatter's idle lanes write).
static size_t bin_ws_bytes(int nb, int64_t n, int lg, int F, int kt2_log2)
{
    const int64_t ncnt = (int64_t)nb * kBinBlocks;
    return align256((size_t)SNAKE_MAX_LEVELS * 4) + 2 * align256((size_t)ncnt * 4) +
           align256((size_t)scan::scan_blocks(ncnt) * 8) + 256 + align256(((size_t)lg << kt2_log2) * F * 16) +
           align256(((size_t)n * lg * 8 + 1) * (F == 4 ? 2 : 1) * 8);
}

static BinPlan make_plan(int L, int F, int log2T, int K, int l0, int lg)
{
    BinPlan bp;
    bp.l0 = l0;
    bp.lg = lg;
    bp.T_log2 = log2T;
    int kt = log2T;
    while ((1 << (kt - log2T)) < K) ++kt;      // padded K*T
    bp.kt2_log2 = kt;
    const int acc_log2 = F == 1 ? 13 : F == 2 ? 12 : 11;   // 2^acc_log2 * F int64 = 64 KB (one accumulator)
    bp.binshift = kt < acc_log2 ? kt : acc_log2;
    bp.nbpl = 1 << (kt - bp.binshift);
    bp.nb = lg * bp.nbpl;
    return bp;
}

int make_grid(const snake_grid_desc *d, int K, Grid &g, const char *fn)
{
    SNAKE_REQUIRE(d != nullptr, SNAKE_ERR_NULL, "%s: grid descriptor is NULL", fn);
    SNAKE_REQUIRE((d->flags & ~(SNAKE_GRID_ALWAYS_HASH | SNAKE_GRID_TABLE_BF16)) == 0u, SNAKE_ERR_INVALID_ARG,
                  "%s: unknown grid flags 0x%x", fn, d->flags);
    SNAKE_REQUIRE(d->n_levels >= 1 && d->n_levels <= SNAKE_MAX_LEVELS, SNAKE_ERR_INVALID_ARG,
                  "%s: n_levels = %d not in [1, %d]", fn, d->n_levels, SNAKE_MAX_LEVELS);
    SNAKE_REQUIRE(d->n_features == 1 || d->n_features == 2 || d->n_features == 4, SNAKE_ERR_UNSUPPORTED,
                  "%s: n_features = %d not in {1, 2, 4}", fn, d->n_features);
    SNAKE_REQUIRE(d->log2_table >= 4 && d->log2_table <= 24, SNAKE_ERR_INVALID_ARG,
                  "%s: log2_table = %d not in [4, 24]", fn, d->log2_table);
    SNAKE_REQUIRE(d->feat_dtype == SNAKE_F32 || d->feat_dtype == SNAKE_BF16, SNAKE_ERR_INVALID_ARG,
                  "%s: bad feat_dtype %d", fn, d->feat_dtype);
    SNAKE_REQUIRE(K >= 1 && K <= 256, SNAKE_ERR_INVALID_ARG, "%s: K = %d not in [1, 256]", fn, K);
    g.K = K;
    g.err = device_error_word();
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

int snake_convert_bf16(const float *src, int64_t n, void *dst, snake_stream_t stream)
{
    SNAKE_REQUIRE(n >= 0 && n % 4 == 0, SNAKE_ERR_INVALID_ARG, "snake_convert_bf16: n = %lld not a multiple of 4",
                  (long long)n);
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(src);
    SNAKE_NOT_NULL(dst);
    SNAKE_ALIGNED(src, 16);
    SNAKE_ALIGNED(dst, 8);
    to_bf16_kernel<<<grid_for(n / 4, 256, 8), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        reinterpret_cast<const float4 *>(src), n / 4, static_cast<uint2 *>(dst));
    return launch_status(__func__);
}

int snake_hashgrid_fwd(const snake_grid_desc *gd, int32_t K, const void *table, const float *pos,
                       const uint8_t *tile_id, const int32_t *sample_idx, int64_t n,
                       const int64_t *n_dev, void *feat, uint32_t *idx_dbg, snake_stream_t stream)
{
    Grid g;
    int rc = make_grid(gd, K, g, __func__);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_hashgrid_fwd: n < 0");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(table);
    SNAKE_NOT_NULL(pos);
    SNAKE_NOT_NULL(feat);
    SNAKE_ALIGNED(table, 16);
    const int F = gd->n_features;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int superchunk = tune(SNAKE_TUNE_HASH_FWD_SUPERCHUNK) * 4096;   // in 256-sample chunks
    const bool bf = gd->feat_dtype == SNAKE_BF16;
    const bool tb = (gd->flags & SNAKE_GRID_TABLE_BF16) != 0;
    if (F == 2) SNAKE_ALIGNED(feat, bf ? 4 : 8);    // one store per sample-level
    // Levels whose slice of one tile fits in a block's LDS are gathered from
    // an LDS copy, the rest through the caches.
    const uint32_t all = g.L == 32 ? 0xffffffffu : (1u << g.L) - 1u;
    uint32_t lds_lv = 0;
    size_t lds_max = 0;
    if (tune(SNAKE_TUNE_HASH_FWD_LDS)) {
        const size_t budget = (size_t)lds_bytes(false) - 256;    // less the kernel's own LDS words
        const size_t esz = (size_t)F * (tb ? 2 : 4);
        for (int l = 0; l < g.L; ++l) {
            const uint64_t side = (uint64_t)g.res[l] + 1;
            const uint64_t entries = ((g.dense_bits >> l) & 1u) ? side * side * side : (uint64_t)g.mask + 1;
            const size_t bytes = (size_t)((entries * esz + 15) / 16 * 16);
            if (bytes <= budget) {
                lds_lv |= 1u << l;
                lds_max = bytes > lds_max ? bytes : lds_max;
            }
        }
    }
    const uint32_t l2_lv = all & ~lds_lv;
    const unsigned grid = grid_for(n * __builtin_popcount(l2_lv), 256, tune(SNAKE_TUNE_HASH_FWD_BLOCKS_PER_CU));
    // at most two 1024-thread blocks fit a CU's wavefront slots
    const int per_cu = (int)((size_t)lds_bytes(true) / (lds_max + 256));
    const unsigned lgrid = grid_for((n + (int64_t)kLdsThreads * kLdsR - 1) / ((int64_t)kLdsThreads * kLdsR) *
                                        kLdsThreads, kLdsThreads, per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
    const float *tf = static_cast<const float *>(table);
    const __hip_bfloat16 *th = static_cast<const __hip_bfloat16 *>(table);
    __hip_bfloat16 *fh = static_cast<__hip_bfloat16 *>(feat);
    float *ff = static_cast<float *>(feat);
#define SNAKE_HG_FWD1(FF, OT, TT, tab, out)                                                                      \
    do {                                                                                                         \
        if (lds_lv)                                                                                              \
            hashgrid_fwd_lds_kernel<FF, OT, TT><<<lgrid, kLdsThreads, lds_max, st>>>(                            \
                g, tab, pos, tile_id, sample_idx, n, n_dev, out, idx_dbg, lds_lv);                               \
        if (l2_lv)                                                                                               \
            hashgrid_fwd_kernel<FF, OT, TT><<<grid, 256, 0, st>>>(g, tab, pos, tile_id, sample_idx, n, n_dev,    \
                                                                  out, idx_dbg, superchunk, l2_lv);              \
    } while (0)
#define SNAKE_HG_FWD(FF)                                                                                         \
    if (tb && bf)                                                                                                \
        SNAKE_HG_FWD1(FF, __hip_bfloat16, __hip_bfloat16, th, fh);                                               \
    else if (tb)                                                                                                 \
        SNAKE_HG_FWD1(FF, float, __hip_bfloat16, th, ff);                                                        \
    else if (bf)                                                                                                 \
        SNAKE_HG_FWD1(FF, __hip_bfloat16, float, tf, fh);                                                        \
    else                                                                                                         \
        SNAKE_HG_FWD1(FF, float, float, tf, ff)
    if (F == 1) {
        SNAKE_HG_FWD(1);
    } else if (F == 2) {
        SNAKE_HG_FWD(2);
    } else {
        SNAKE_HG_FWD(4);
    }
#undef SNAKE_HG_FWD
#undef SNAKE_HG_FWD1
    return launch_status(__func__);
}

size_t snake_hashgrid_bwd_workspace_bytes(const snake_grid_desc *gd, int32_t K, int64_t n,
                                          int32_t levels_per_pass)
{
    Grid g;
    if (make_grid(gd, K, g, __func__) || n < 0) return 0;
    const int lg = levels_per_pass < 1 ? 1 : (levels_per_pass > g.L ? g.L : levels_per_pass);
    const BinPlan bp = make_plan(g.L, gd->n_features, gd->log2_table, K, 0, lg);
    return bin_ws_bytes(bp.nb, n, lg, gd->n_features, bp.kt2_log2);
}

int snake_hashgrid_bwd(const snake_grid_desc *gd, int32_t K, const float *pos, const uint8_t *tile_id,
                       const int32_t *sample_idx, int64_t n, const int64_t *n_dev, const float *dfeat,
                       float *dtable, void *workspace, size_t workspace_bytes, snake_stream_t stream)
{
    Grid g;
    int rc = make_grid(gd, K, g, __func__);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_hashgrid_bwd: n < 0");
    SNAKE_REQUIRE((int64_t)K << gd->log2_table <= ((int64_t)1 << 28), SNAKE_ERR_INVALID_ARG,
                  "snake_hashgrid_bwd: K * T exceeds 2^28 slots per level");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(pos);
    SNAKE_NOT_NULL(dfeat);
    SNAKE_NOT_NULL(dtable);
    const int F = gd->n_features;
    SNAKE_ALIGNED(dfeat, 4 * F);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (workspace == nullptr) {
        const unsigned grid = grid_for(n * g.L, 256, 16);
        if (F == 1)
            hashgrid_bwd_kernel<1><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
        else if (F == 2)
            hashgrid_bwd_kernel<2><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
        else
            hashgrid_bwd_kernel<4><<<grid, 256, 0, st>>>(g, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable);
        return launch_status(__func__);
    }
    SNAKE_ALIGNED(workspace, 256);
    SNAKE_REQUIRE(n * 8 <= (int64_t)INT32_MAX, SNAKE_ERR_INVALID_ARG,
                  "snake_hashgrid_bwd: n = %lld too large for the binned adjoint (n * 8 < 2^31)", (long long)n);
    {
        const BinPlan b1 = make_plan(g.L, F, gd->log2_table, K, 0, 1);
        SNAKE_REQUIRE(b1.nb <= kMaxBins && scatter_lds_bytes(b1.nb, b1.nbpl, F) <= kScatterLds, SNAKE_ERR_UNSUPPORTED,
                      "snake_hashgrid_bwd: K * T = %lld slots per level is too many for the binned adjoint "
                      "(pass workspace = NULL for the atomic form)", (long long)K << gd->log2_table);
    }
    // largest level group whose items fit the workspace (and the tuned cap)
    const int nblk = tune(SNAKE_TUNE_BIN_BLOCKS);
    const int lg_cap = tune(SNAKE_TUNE_BIN_LEVELS_PER_PASS);
    int lg = 0;
    for (int cand = lg_cap > 0 && lg_cap < g.L ? lg_cap : g.L; cand >= 1; --cand) {
        const BinPlan bp = make_plan(g.L, F, gd->log2_table, K, 0, cand);
        // item offsets are int32: a pass holds fewer than 2^31 items
        if (bp.nb <= kMaxBins && scatter_lds_bytes(bp.nb, bp.nbpl, F) <= kScatterLds &&
            n * cand * 8 <= (int64_t)INT32_MAX && bin_ws_bytes(bp.nb, n, cand, F, bp.kt2_log2) <= workspace_bytes) {
            lg = cand;
            break;
        }
    }
    SNAKE_REQUIRE(lg >= 1, SNAKE_ERR_WORKSPACE, "snake_hashgrid_bwd: workspace needs at least %zu bytes",
                  snake_hashgrid_bwd_workspace_bytes(gd, K, n, 1));
    {
        // as few passes as that allows, with their levels spread evenly
        // (each pass re-reads every sample's position)
        const int npass = (g.L + lg - 1) / lg;
        lg = (g.L + npass - 1) / npass;
    }
    // per-level scale of the fixed-point sums, from the largest |dfeat|
    uint32_t *lmax = static_cast<uint32_t *>(workspace);
    unsigned int *err = device_error_word();
    // the per-level maxima are taken by each pass's count kernel
    zero_u32_kernel<<<1, 64, 0, st>>>(lmax, g.L);
    for (int l0 = 0; l0 < g.L; l0 += lg) {
        const int lgp = l0 + lg <= g.L ? lg : g.L - l0;
        const BinPlan bp = make_plan(g.L, F, gd->log2_table, K, l0, lgp);
        const int64_t ncnt = (int64_t)bp.nb * nblk;
        char *p = static_cast<char *>(workspace) + align256((size_t)SNAKE_MAX_LEVELS * 4);
        BinWs w;
        w.lmax = lmax;
        w.counts = reinterpret_cast<int32_t *>(p);
        p += align256((size_t)ncnt * 4);
        w.offsets = reinterpret_cast<int32_t *>(p);
        p += align256((size_t)ncnt * 4);
        w.bsum = reinterpret_cast<int64_t *>(p);
        p += align256((size_t)scan::scan_blocks(ncnt) * 8);
        w.n_items = reinterpret_cast<int64_t *>(p);
        p += 256;
        const int64_t n_acc = ((int64_t)lgp << bp.kt2_log2) * F * 2;
        w.acc64 = reinterpret_cast<unsigned long long *>(p);
        p += align256((size_t)n_acc * 8);
        w.items = reinterpret_cast<unsigned long long *>(p);
        w.item_cap = n * lgp * 8;
        const unsigned rgrid = (unsigned)(kReducePerCU * num_cus());
        const unsigned zgrid = grid_for(n_acc, 256, 8);
        const unsigned cgrid = grid_for(((int64_t)lgp * K << gd->log2_table) * F, 256, 8);
#define SNAKE_BIN_PASS(FF)                                                                                 \
    zero_u64_kernel<<<zgrid, 256, 0, st>>>(w.acc64, n_acc);                                                \
    bin_count_kernel<FF><<<nblk, 256, 0, st>>>(g, bp, pos, tile_id, sample_idx, n, n_dev, dfeat, w.lmax,     \
                                               w.counts);                                                  \
    scan::launch_scan(w.counts, ncnt, w.bsum, w.offsets, 1, nullptr, w.item_cap, w.n_items, err, st);   \
    bin_scatter_kernel<FF><<<nblk, ScatterShape<FF>::threads, scatter_lds_bytes(bp.nb, bp.nbpl, FF), st>>>( \
        g, bp, pos, tile_id, sample_idx, n, n_dev, dfeat, w.offsets, w.counts, w.lmax, w.items, w.item_cap); \
    bin_reduce_kernel<FF><<<rgrid, kReduceThreads, 0, st>>>(bp, w.offsets, nblk, w.n_items, w.items, w.lmax, w.acc64); \
    bin_convert_kernel<FF><<<cgrid, 256, 0, st>>>(bp, g.L, w.acc64, w.lmax, K, dtable)
        if (F == 1) {
            SNAKE_BIN_PASS(1);
        } else if (F == 2) {
            SNAKE_BIN_PASS(2);
        } else {
            SNAKE_BIN_PASS(4);
        }
#undef SNAKE_BIN_PASS
    }
    return launch_status(__func__);
}

}  // extern "C"
