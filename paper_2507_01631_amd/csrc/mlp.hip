// Density and colour networks of a tile NeRF (Sec. 4.1) on CDNA4 matrix cores.
//
// Shapes are fixed by the architecture: density 32 -> 64 -> 16 (ReLU hidden,
// sigma = exp(o_0), embedding o_1..o_15), colour [o_1..o_15, view, (sun)] ->
// 64 (-> 64) -> 3|4, no biases.
//
// Every layer is a 16-sample tile multiplied on MFMA: weights are the A
// operand (output units x inputs), activations the B operand (inputs x 16
// samples), so a layer's output (lane (i, q) holds rows 4q..4q+3 of sample i)
// is directly the next layer's B operand once the weight fragments in LDS
// carry the matching K permutation.  FP32 form: v_mfma_f32_16x16x4_f32.
// BF16 form: v_mfma_f32_16x16x32_bf16 (K=16 layers: 16x16x16) with FP32
// accumulation; inputs, weights and hidden activations rounded RNE to bf16.
//
// The adjoint recomputes activations from the features (or reads them back
// when the forward stored them), runs the transposed chain, and accumulates
// weight gradients with MFMA over samples (K = samples) after an LDS
// transpose: per wavefront in the FP32 form, split across the block's four
// wavefronts in the BF16 form (which then fits two wavefronts per SIMD).
// Per-block partial sums are reduced in a fixed order by a second kernel.
#include <type_traits>

#include "common.h"

namespace snake {

struct MlpArgs {
    int L, F, n_feat;       // encoding levels, features per level, L*F
    int n_dir, CL, CO;      // directions (3|6), colour hidden layers (1|2), colour outputs (3|4)
    int cin_real;           // 15 + n_dir
    int32_t off[5];         // offsets of D1, D2, C1, C2, CO in the packed weights
    int32_t P;              // packed parameter count
    int32_t R;              // rows of view / sun (ray ids must be below)
    unsigned int *err;      // device error word
    int K;                  // NeRF tiles, each with its own weight set
    const int64_t *tile_start;  // [K+2] sample groups per tile (NULL: one group)
    int shared_colour;      // 1: density nets per tile, one colour net for all
    int32_t Pd;             // density parameters of one set (D1 + D2)
};

// The BF16 pipelined adjoint (mlp_bwd_pipe_kernel<P_BF16, ...>) is compiled in
// a translation unit of its own, mlp_bwd16.hip (this file with SNAKE_MLP_BWD16
// defined), whose scheduler minimises registers: the kernel holds about 400
// values at two wavefronts per SIMD, and fewer spills pay more than the
// latency the other schedule hides.  cl: colour hidden layers; feat_bf16:
// features stored as BF16 (else FP32).
void launch_bwd_pipe_bf16(const MlpArgs &a, int cl, bool feat_bf16, unsigned grid, const float *w, const void *feat,
                          int64_t feat_ld, const float *view, const float *sun, const int32_t *ray_id,
                          const int32_t *sidx, int64_t n, const int64_t *n_dev, const float *dsigma,
                          const float *drgb, float *dfeat, float *partial, const void *frag, hipStream_t st);

namespace {

#ifdef SNAKE_MLP_BWD16
constexpr bool kBwd16Unit = true;
#else
constexpr bool kBwd16Unit = false;
#endif

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;   // 4 wavefronts
constexpr int kMaxBwdBlocks = 512;

enum Prec { P_F32 = 0, P_BF16 = 1 };
enum Mat { M_D1 = 0, M_D2, M_C1, M_C2, M_CO };



// Base pointers of tile k's density and colour weights, so that
// wd + off[0..1] and wc + off[2..4] address its matrices.  Per-tile sets are
// [K][P]; with a shared colour net the layout is [K][Pd] then one colour set.
__host__ __device__ inline void tile_weights(const MlpArgs &a, const float *w, int k, const float *&wd,
                                             const float *&wc)
{
    if (a.shared_colour) {
        wd = w + (int64_t)k * a.Pd;
        wc = w + (int64_t)a.K * a.Pd - a.Pd;
    } else {
        wd = wc = w + (int64_t)k * a.P;
    }
}

constexpr int kMaxMlpTiles = 16;
const int64_t kNoTable = 0;   // stands in for tile_start in size queries

// Work units of 64 samples (one 16-sample matrix tile per wavefront) that
// never straddle two NeRF tiles.  Group k < K is samples [ts[k], ts[k+1]) of
// the call; group K holds samples whose tile id was invalid (dropped).  The
// bounds are clamped to be non-decreasing and within [0, ne], so a corrupt
// table cannot send a unit out of range.  Every thread of a block sees the
// same units, so branches on them are block-uniform.
struct UnitTable {
    int64_t ts[kMaxMlpTiles + 2];
    int64_t ub[kMaxMlpTiles + 2];   // first unit of each group; ub[K+1] = total
};

__device__ void setup_units(UnitTable &U, const MlpArgs &a, int64_t ne)
{
    if (threadIdx.x == 0) {
        int64_t prev = 0, units = 0;
        for (int k = 0; k <= a.K + 1; ++k) {
            int64_t v;
            if (a.tile_start)
                v = a.tile_start[k];
            else
                v = k == 0 ? 0 : ne;
            v = v < prev ? prev : (v > ne ? ne : v);
            if (k > 0) units += (v - prev + 63) / 64;
            U.ts[k] = v;
            U.ub[k] = units;        // ub[k] = units of groups < k
            prev = v;
        }
    }
    __syncthreads();
}

// Group, first sample and end of unit u.
__device__ __forceinline__ void locate(const UnitTable &U, int K, int64_t u, int &k, int64_t &s0, int64_t &s1)
{
    k = 0;
    while (k < K && u >= U.ub[k + 1]) ++k;
    s0 = U.ts[k] + 64 * (u - U.ub[k]);
    s1 = U.ts[k + 1];
}

// Padded weight value: D1 [64][32], D2 [16][64], C1 [64][32] whose column p
// is o_p (p < 16, column 0 = sigma logit is 0) or direction p-16, C2 [64][64],
// CO [16][64] (rows >= CO are 0).
__device__ __forceinline__ float wval(const float *w, const MlpArgs &a, int mat, int r, int c)
{
    switch (mat) {
    case M_D1:
        return w[a.off[0] + r * 32 + c];
    case M_D2:
        return w[a.off[1] + r * 64 + c];
    case M_C1:
        if (c >= 1 && c < 16) return w[a.off[2] + r * a.cin_real + (c - 1)];
        if (c >= 16 && c < 16 + a.n_dir) return w[a.off[2] + r * a.cin_real + 15 + (c - 16)];
        return 0.0f;
    case M_C2:
        return w[a.off[3] + r * 64 + c];
    default:
        return r < a.CO ? w[a.off[4] + r * 64 + c] : 0.0f;
    }
}

template <int PREC>
struct FragT {
    typedef float T;
};
template <>
struct FragT<P_BF16> {
    typedef __bf16 T;
};

// Fill the A-operand fragments of an MO x MI layer (W or W^T of `mat`).
template <int PREC, int MO, int MI>
__device__ void build_frag(typename FragT<PREC>::T *dst, const float *w, const MlpArgs &a, int mat,
                           bool transposed)
{
    for (int e = threadIdx.x; e < MO * MI; e += blockDim.x) {
        int row, col;
        if (PREC == P_F32) {
            const int r = e & 3, lane = (e >> 2) & 63, blk = e >> 8;
            const int to = blk / (MI / 16), ti = blk % (MI / 16);
            row = 16 * to + (lane & 15);
            col = 16 * ti + 4 * (lane >> 4) + r;
        } else if (MI % 32 == 0) {
            const int k = e & 7, lane = (e >> 3) & 63, blk = e >> 9;
            const int to = blk / (MI / 32), u = blk % (MI / 32), q = lane >> 4;
            row = 16 * to + (lane & 15);
            col = 32 * u + (k < 4 ? 4 * q + k : 16 + 4 * q + (k - 4));
        } else {
            const int k = e & 3, lane = (e >> 2) & 63, to = e >> 8;
            row = 16 * to + (lane & 15);
            col = 4 * (lane >> 4) + k;
        }
        const float v = transposed ? wval(w, a, mat, col, row) : wval(w, a, mat, row, col);
        dst[e] = (typename FragT<PREC>::T)v;
    }
}

// y[MO/16][4] = W (MO x MI) . x[MI/16][4] for one 16-sample tile.
template <int PREC, int MO, int MI>
__device__ __forceinline__ void apply(const typename FragT<PREC>::T *frag, const float (&x)[MI / 16][4],
                                      float (&y)[MO / 16][4])
{
    const int lane = lane_id();
    if constexpr (PREC == P_F32) {
        const f4 *fr = reinterpret_cast<const f4 *>(frag);
#pragma unroll
        for (int to = 0; to < MO / 16; ++to) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ti = 0; ti < MI / 16; ++ti) {
                const f4 av = fr[(to * (MI / 16) + ti) * 64 + lane];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], x[ti][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], x[ti][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], x[ti][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], x[ti][3], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) y[to][r] = acc[r];
        }
    } else if constexpr (MI % 32 == 0) {
        const bf8 *fr = reinterpret_cast<const bf8 *>(frag);
        bf8 b[MI / 32];
#pragma unroll
        for (int u = 0; u < MI / 32; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                b[u][r] = (__bf16)x[2 * u][r];
                b[u][4 + r] = (__bf16)x[2 * u + 1][r];
            }
#pragma unroll
        for (int to = 0; to < MO / 16; ++to) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < MI / 32; ++u)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[(to * (MI / 32) + u) * 64 + lane], b[u], acc, 0,
                                                             0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) y[to][r] = acc[r];
        }
    } else {
        static_assert(MI == 16, "K=16 layers only");
        const s4 *fr = reinterpret_cast<const s4 *>(frag);
        bf4 bb;
#pragma unroll
        for (int r = 0; r < 4; ++r) bb[r] = (__bf16)x[0][r];
        const s4 b = __builtin_bit_cast(s4, bb);
#pragma unroll
        for (int to = 0; to < MO / 16; ++to) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fr[to * 64 + lane], b, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) y[to][r] = acc[r];
        }
    }
}

// max(v, 0) as an integer maximum of the bits (a negative float is a
// negative integer): one instruction, where fmaxf first quiets a possible
// signalling NaN with a second one.  -0 becomes +0.
// A BF16 layer with K = 32 whose operand is given as four words of two bf16
// each (the bf8 operand apply() would pack from x[2][4]); the same products.
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
template <int MO>
__device__ __forceinline__ void apply_bf16_words(const __bf16 *frag, const uint32_t (&w)[4], float (&y)[MO / 16][4])
{
    const int lane = lane_id();
    const bf8 *fr = reinterpret_cast<const bf8 *>(frag);
    const bf8 b = __builtin_bit_cast(bf8, u4v{w[0], w[1], w[2], w[3]});
#pragma unroll
    for (int to = 0; to < MO / 16; ++to) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[to * 64 + lane], b, acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) y[to][r] = acc[r];
    }
}

template <int T>
__device__ __forceinline__ void relu(float (&v)[T][4])
{
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = __builtin_bit_cast(int, v[t][r]);
            v[t][r] = __builtin_bit_cast(float, b > 0 ? b : 0);
        }
}

template <int T>
__device__ __forceinline__ void relu_mask(float (&d)[T][4], const float (&act)[T][4])
{
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) d[t][r] = act[t][r] > 0.0f ? d[t][r] : 0.0f;
}

__device__ __forceinline__ float load_f(const float *p) { return *p; }
__device__ __forceinline__ float load_f(const __hip_bfloat16 *p) { return __bfloat162float(*p); }

__device__ __forceinline__ float2 load_pair(const float *p) { return *reinterpret_cast<const float2 *>(p); }
__device__ __forceinline__ float2 load_pair(const __hip_bfloat16 *p)
{
    const uint32_t w = *reinterpret_cast<const uint32_t *>(p);
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

// Density input rows 0..31 (row p = level p/F, feature p%F; rows >= L*F are 0).
template <typename FT>
__device__ __forceinline__ void load_features(const FT *feat, int64_t ld, int64_t s, bool valid,
                                              const MlpArgs &a, float (&x)[2][4])
{
    const int q = lane_id() >> 4;
    if (a.F == 2) {             // rows 2m, 2m+1 are the two features of level m: one load
        // level 8t + 2q + h: a per-lane base and uniform level offsets
        const FT *base = feat + ((int64_t)(2 * q) * ld + s) * 2;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = 16 * t + 4 * q + 2 * h;
                float2 v = make_float2(0.0f, 0.0f);
                if (valid && p < a.n_feat) v = load_pair(base + (int64_t)(8 * t + h) * ld * 2);
                x[t][2 * h] = v.x;
                x[t][2 * h + 1] = v.y;
            }
        return;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * t + 4 * q + r;
            float v = 0.0f;
            if (valid && p < a.n_feat) {
                const int lvl = p / a.F, f = p - lvl * a.F;
                v = load_f(feat + ((int64_t)lvl * ld + s) * a.F + f);
            }
            x[t][r] = v;
        }
}

// Raw feature words of one lane for the pipelined forward (F == 2): the
// loads issue back to back and nothing reads their results until the unit is
// computed, so they stay in flight meanwhile.  Every lane loads from a valid
// address (row 0 of the first sample when its own rows are not wanted).
template <typename FT>
struct RawFeat;
template <>
struct RawFeat<__hip_bfloat16> {
    uint32_t w[2][2];
    __device__ void load(const __hip_bfloat16 *p, int t, int h) { w[t][h] = *reinterpret_cast<const uint32_t *>(p); }
    __device__ float2 get(int t, int h) const
    {
        return make_float2(__uint_as_float(w[t][h] << 16), __uint_as_float(w[t][h] & 0xffff0000u));
    }
};
template <>
struct RawFeat<float> {
    float2 w[2][2];
    __device__ void load(const float *p, int t, int h) { w[t][h] = *reinterpret_cast<const float2 *>(p); }
    __device__ float2 get(int t, int h) const { return w[t][h]; }
};

template <typename FT>
__device__ __forceinline__ void issue_features(const FT *feat, int64_t ld, int64_t s, bool valid, const MlpArgs &a,
                                               RawFeat<FT> &raw, uint32_t &use)
{
    const int q = lane_id() >> 4;
    use = 0u;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lvl = 8 * t + 2 * q + h;           // rows 2 lvl, 2 lvl + 1: the level's two features
            const bool u = valid && 2 * lvl < a.n_feat;
            raw.load(feat + (u ? (int64_t)lvl * ld + s : 0) * 2, t, h);
            use |= (u ? 1u : 0u) << (2 * t + h);
        }
}

template <typename FT>
__device__ __forceinline__ void take_features(const RawFeat<FT> &raw, uint32_t use, bool ok, float (&x)[2][4])
{
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool u = ok && ((use >> (2 * t + h)) & 1u);
            const float2 v = raw.get(t, h);
            x[t][2 * h] = u ? v.x : 0.0f;
            x[t][2 * h + 1] = u ? v.y : 0.0f;
        }
}

// Colour-input directions of one lane (rows 16..31: view xyz, sun xyz, then
// zeros), loaded from valid addresses without branches; mask bit r says
// whether row 4q + r is a direction.
__device__ __forceinline__ void issue_dirs(const float *view, const float *sun, int64_t ray, const MlpArgs &a,
                                           float (&c)[4], uint32_t &mask)
{
    const int q = lane_id() >> 4;
    mask = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 4 * q + r;
        const bool from_view = k < 3, from_sun = k >= 3 && k < a.n_dir && sun != nullptr;
        const uintptr_t pv = reinterpret_cast<uintptr_t>(view + (from_view ? 3 * ray + k : 0));
        const uintptr_t ps = reinterpret_cast<uintptr_t>(sun + (from_sun ? 3 * ray + (k - 3) : 0));
        c[r] = *reinterpret_cast<const float *>(from_sun ? ps : pv);
        mask |= (from_view || from_sun ? 1u : 0u) << r;
    }
}

// Colour input rows 16..31: view xyz, sun xyz (n_dir == 6), then zeros.
__device__ __forceinline__ void load_dirs(const float *view, const float *sun, int64_t ray, bool valid,
                                          const MlpArgs &a, float (&c)[4])
{
    const int q = lane_id() >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 4 * q + r;
        float v = 0.0f;
        if (valid) {
            if (k < 3)
                v = view[3 * ray + k];
            else if (k < a.n_dir)
                v = sun[3 * ray + (k - 3)];
        }
        c[r] = v;
    }
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

template <int PREC, int CL>
struct Layout {
    typedef typename FragT<PREC>::T T;
    // forward fragments
    static constexpr int D1 = 0;
    static constexpr int D2 = D1 + 64 * 32;
    static constexpr int C1 = D2 + 16 * 64;
    static constexpr int C2 = C1 + 64 * 32;
    static constexpr int CO = C2 + (CL == 2 ? 64 * 64 : 0);
    static constexpr int FWD = CO + 16 * 64;
    // adjoint (transposed) fragments
    static constexpr int COT = FWD;
    static constexpr int C2T = COT + 64 * 16;
    static constexpr int C1T = C2T + (CL == 2 ? 64 * 64 : 0);
    static constexpr int D2T = C1T + 16 * 64;
    static constexpr int D1T = D2T + 64 * 16;
    static constexpr int ALL = D1T + 32 * 64;
};

template <int PREC, int CL>
__device__ void build_forward(typename FragT<PREC>::T *lds, const float *wd, const float *wc, const MlpArgs &a)
{
    typedef Layout<PREC, CL> Lt;
    build_frag<PREC, 64, 32>(lds + Lt::D1, wd, a, M_D1, false);
    build_frag<PREC, 16, 64>(lds + Lt::D2, wd, a, M_D2, false);
    build_frag<PREC, 64, 32>(lds + Lt::C1, wc, a, M_C1, false);
    if (CL == 2) build_frag<PREC, 64, 64>(lds + Lt::C2, wc, a, M_C2, false);
    build_frag<PREC, 16, 64>(lds + Lt::CO, wc, a, M_CO, false);
}

// Forward of one 16-sample tile; keeps every activation.
template <int PREC, int CL>
struct Acts {
    float x[2][4], h1[4][4], o[1][4], cin[2][4], g1[4][4], g2[4][4], out[1][4];
};

template <int PREC, int CL>
__device__ __forceinline__ void forward_tile(const typename FragT<PREC>::T *lds, Acts<PREC, CL> &A)
{
    typedef Layout<PREC, CL> Lt;
    apply<PREC, 64, 32>(lds + Lt::D1, A.x, A.h1);
    relu(A.h1);
    apply<PREC, 16, 64>(lds + Lt::D2, A.h1, A.o);
#pragma unroll
    for (int r = 0; r < 4; ++r) A.cin[0][r] = A.o[0][r];
    apply<PREC, 64, 32>(lds + Lt::C1, A.cin, A.g1);
    relu(A.g1);
    if constexpr (CL == 2) {
        apply<PREC, 64, 64>(lds + Lt::C2, A.g1, A.g2);
        relu(A.g2);
        apply<PREC, 16, 64>(lds + Lt::CO, A.g2, A.out);
    } else {
        apply<PREC, 16, 64>(lds + Lt::CO, A.g1, A.out);
    }
}

// Stored activations of one sample: h1 [64] | o [16] | g1 [64] | g2 [64] (two
// colour layers only) | out [16]; element 16t + 4q + r of an array is row
// 4q + r of its tile t, so each lane moves 16-byte pieces.
template <int CL>
struct ActLayout {
    static constexpr int H1 = 0, O = 64, G1 = 80, G2 = 144;
    static constexpr int OUT = CL == 2 ? 208 : 144;
    static constexpr int W = OUT + 16;
};

template <int T>
__device__ __forceinline__ void act_put(float *row, int base, const float (&v)[T][4])
{
    const int q = lane_id() >> 4;
#pragma unroll
    for (int t = 0; t < T; ++t)
        *reinterpret_cast<f4 *>(row + base + 16 * t + 4 * q) = f4{v[t][0], v[t][1], v[t][2], v[t][3]};
}

template <int T>
__device__ __forceinline__ void act_get(const float *row, int base, float (&v)[T][4])
{
    const int q = lane_id() >> 4;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const f4 u = *reinterpret_cast<const f4 *>(row + base + 16 * t + 4 * q);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[t][r] = u[r];
    }
}

template <int PREC, int CL>
__device__ __forceinline__ void store_acts(float *row, const Acts<PREC, CL> &A)
{
    typedef ActLayout<CL> AL;
    act_put(row, AL::H1, A.h1);
    act_put(row, AL::O, A.o);
    act_put(row, AL::G1, A.g1);
    if constexpr (CL == 2) act_put(row, AL::G2, A.g2);
    act_put(row, AL::OUT, A.out);
}

template <int PREC, int CL>
__device__ __forceinline__ void load_acts(const float *row, Acts<PREC, CL> &A)
{
    typedef ActLayout<CL> AL;
    act_get(row, AL::H1, A.h1);
    act_get(row, AL::O, A.o);
#pragma unroll
    for (int r = 0; r < 4; ++r) A.cin[0][r] = A.o[0][r];
    act_get(row, AL::G1, A.g1);
    if constexpr (CL == 2) act_get(row, AL::G2, A.g2);
    act_get(row, AL::OUT, A.out);
}

// Per-lane inputs of one 16-sample tile of the adjoint: where they are, and
// the values.
struct BwdIdx {
    int64_t s, si;
    int ray;
    bool in_range;
};

struct BwdIn {
    bool valid;
    float x[2][4], dirs[4], dsig, dr[3];
};

template <int PREC, int CL, typename FT, bool STORE>
__global__ __launch_bounds__(kBlock) void mlp_fwd_kernel(MlpArgs a, const float *__restrict__ w,
                                                         const FT *__restrict__ feat,
                                                         const float *__restrict__ view,
                                                         const float *__restrict__ sun,
                                                         const int32_t *__restrict__ ray_id,
                                                         const int32_t *__restrict__ sidx, int64_t n,
                                                         const int64_t *__restrict__ n_dev,
                                                         float *__restrict__ sigma, float *__restrict__ rgb,
                                                         float *__restrict__ act)
{
    typedef Layout<PREC, CL> Lt;
    __shared__ __attribute__((aligned(16))) typename Lt::T lds[Lt::FWD];
    __shared__ UnitTable U;
    const int64_t ne = effective_n(n, n_dev);
    setup_units(U, a, ne);
    const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
    const int64_t total = U.ub[a.K + 1];
    int cur = -1;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        int k;
        int64_t s0, s1;
        locate(U, a.K, u, k, s0, s1);
        const int64_t s = s0 + 16 * wv + i;
        const bool valid = s < s1;
        if (k == a.K) {                                      // invalid tile id: dropped
            if (q == 0 && valid) {
                sigma[s] = 0.0f;
                rgb[3 * s] = rgb[3 * s + 1] = rgb[3 * s + 2] = 0.0f;
            }
            continue;
        }
        if (k != cur) {                                      // block-uniform
            __syncthreads();
            const float *wd, *wc;
            tile_weights(a, w, k, wd, wc);
            build_forward<PREC, CL>(lds, wd, wc, a);
            __syncthreads();
            cur = k;
        }
        const int64_t si = valid ? (sidx ? sidx[s] : s) : 0;
        Acts<PREC, CL> A;
        int64_t ray = valid ? ray_id[si] : 0;
        const bool ok = valid && ray >= 0 && ray < a.R;     // a bad ray id drops the sample
        if (valid && !ok && q == 0 && a.err) atomicOr(a.err, (unsigned)SNAKE_DEVERR_RAY_ID);
        ray = ok ? ray : 0;
        load_features(feat, n, s, ok, a, A.x);
        load_dirs(view, sun, ray, ok, a, A.cin[1]);
        forward_tile<PREC, CL>(lds, A);
        if constexpr (STORE) {
            if (ok) store_acts<PREC, CL>(act + s * ActLayout<CL>::W, A);
        }
        if (q == 0 && valid && !ok) {
            sigma[s] = 0.0f;
            rgb[3 * s] = rgb[3 * s + 1] = rgb[3 * s + 2] = 0.0f;
        } else if (q == 0 && valid) {
            sigma[s] = expf(A.o[0][0]);
            if (a.CO == 3) {
#pragma unroll
                for (int c = 0; c < 3; ++c) rgb[3 * s + c] = sigmoidf(A.out[0][c]);
            } else {
                const float vis = sigmoidf(A.out[0][3]);
#pragma unroll
                for (int c = 0; c < 3; ++c) rgb[3 * s + c] = sigmoidf(A.out[0][c]) * vis;
            }
        }
    }
}

template <int PREC, int CL, typename FT, bool STORE>
__global__ __launch_bounds__(kBlock) void mlp_fwd_pipe_kernel(MlpArgs a, const float *__restrict__ w,
                                                         const FT *__restrict__ feat,
                                                         const float *__restrict__ view,
                                                         const float *__restrict__ sun,
                                                         const int32_t *__restrict__ ray_id, int64_t n,
                                                         const int64_t *__restrict__ n_dev,
                                                         float *__restrict__ sigma, float *__restrict__ rgb,
                                                         float *__restrict__ act)
{
    typedef Layout<PREC, CL> Lt;
    __shared__ __attribute__((aligned(16))) typename Lt::T lds[Lt::FWD];
    __shared__ UnitTable U;
    const int64_t ne = effective_n(n, n_dev);
    setup_units(U, a, ne);
    const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
    const int64_t total = U.ub[a.K + 1];
    // Software pipeline (F == 2, no index list).  Unit u's ray ids and
    // features are loaded one unit ahead, at the start of the previous unit
    // of this block; its directions (which need the ray ids) at the end of
    // that unit.  Loads issue back to back and no result is read before the
    // layer that needs it, so they stay in flight while a unit is computed.
    struct In {
        int64_t s;
        int k;
        bool valid;
        uint32_t use, dmask;
        int32_t ray;
        RawFeat<FT> raw;
        float dirs[4];
    };
    // Addressing that does not change from unit to unit, set up once: the
    // level slices of this lane's four feature rows (rows 2 lvl, 2 lvl + 1
    // of level lvl = 8t + 2q + h; slice 0 for rows past the input), the
    // sources of its four direction rows (view or sun, 3 floats per ray; a
    // row that is neither reads view[0]), and its output word (lane q = 0:
    // sigma, q = 1..3: colour channel q-1).
    const FT *fb[2][2];
    uint32_t fuse = 0u;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lvl = 8 * t + 2 * q + h;
            const bool u = 2 * lvl < a.n_feat;
            fb[t][h] = feat + (u ? (int64_t)lvl * n : 0) * 2;
            fuse |= (u ? 1u : 0u) << (2 * t + h);
        }
    const float *db[4];
    uint32_t dm = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int kd = 4 * q + r;
        const bool from_view = kd < 3, from_sun = kd >= 3 && kd < a.n_dir && sun != nullptr;
        db[r] = from_sun ? sun + (kd - 3) : view + (from_view ? kd : 0);
        dm |= (from_view || from_sun ? 1u : 0u) << r;
    }
    float *const ob = q == 0 ? sigma : rgb + (q - 1);
    const int64_t ostride = q == 0 ? 1 : 3;
    auto issue = [&](int64_t u, In &in) {
        int64_t s0, s1;
        locate(U, a.K, u, in.k, s0, s1);
        in.s = s0 + 16 * wv + i;
        in.valid = in.s < s1;
        in.ray = ray_id[in.valid ? in.s : s0];               // a sample that exists
        // every lane loads from a valid address; unwanted rows are masked
        const int64_t se = in.valid ? in.s : 0;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) in.raw.load(fb[t][h] + se * 2, t, h);
        in.use = in.valid ? fuse : 0u;
    };
    auto issue_dirs_of = [&](In &in) {
        const bool ok = in.valid && in.k < a.K && in.ray >= 0 && in.ray < a.R;
        const int64_t r3 = 3 * (int64_t)(ok ? in.ray : 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) in.dirs[r] = db[r][((dm >> r) & 1u) ? r3 : 0];
        in.dmask = dm;
    };
    int cur = -1;
    // one unit: compute `in`, loading unit u + grid into `nx` meanwhile (two
    // buffers used alternately, so no loaded value is copied before use)
    auto step = [&](int64_t u, In &in, In &nx) {
        const bool more = u + gridDim.x < total;
        if (more) issue(u + gridDim.x, nx);
        const int64_t s = in.s;
        const bool valid = in.valid && in.k < a.K;
        const bool ok = valid && in.ray >= 0 && in.ray < a.R;   // a bad ray id drops the sample
        if (valid && !ok && q == 0 && a.err) atomicOr(a.err, (unsigned)SNAKE_DEVERR_RAY_ID);
        if (in.k == a.K) {                                   // invalid tile id: dropped
            if (in.valid) ob[s * ostride] = 0.0f;
            if (more) issue_dirs_of(nx);
            return;
        }
        if (in.k != cur) {                                   // block-uniform
            __syncthreads();
            const float *wd, *wc;
            tile_weights(a, w, in.k, wd, wc);
            build_forward<PREC, CL>(lds, wd, wc, a);
            __syncthreads();
            cur = in.k;
        }
        Acts<PREC, CL> A;
        // keep the scheduler from reading loaded values before their layer
        // (the wait for a load sits at its first use)
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (PREC == P_BF16 && std::is_same<FT, __hip_bfloat16>::value) {
            // BF16 features are already the first layer's operand: lane
            // (i, q) holds rows 4q..4q+3 and 16+4q..16+4q+3 of sample i, the
            // four feature-pair words it loaded, in that order
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    w[2 * t + h] = ok && ((in.use >> (2 * t + h)) & 1u) ? in.raw.w[t][h] : 0u;
            apply_bf16_words<64>(lds + Lt::D1, w, A.h1);
        } else {
            take_features<FT>(in.raw, in.use, ok, A.x);
            apply<PREC, 64, 32>(lds + Lt::D1, A.x, A.h1);
        }
        relu(A.h1);
        apply<PREC, 16, 64>(lds + Lt::D2, A.h1, A.o);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            A.cin[0][r] = A.o[0][r];
            A.cin[1][r] = ok && ((in.dmask >> r) & 1u) ? in.dirs[r] : 0.0f;
        }
        apply<PREC, 64, 32>(lds + Lt::C1, A.cin, A.g1);
        relu(A.g1);
        if constexpr (CL == 2) {
            apply<PREC, 64, 64>(lds + Lt::C2, A.g1, A.g2);
            relu(A.g2);
            apply<PREC, 16, 64>(lds + Lt::CO, A.g2, A.out);
        } else {
            apply<PREC, 16, 64>(lds + Lt::CO, A.g1, A.out);
        }
        if constexpr (STORE) {
            if (ok) store_acts<PREC, CL>(act + s * ActLayout<CL>::W, A);
        }
        // The four lanes of a sample share its outputs: lane q = 0 writes
        // sigma = exp(o_0), lane q = 1..3 colour channel q-1 (its logit read
        // from lane q = 0), so each lane evaluates one exponential.
        {
            // every lane takes part in every shuffle (a lane reading from an
            // inactive one would get 0), so they come first, unconditionally
            const float f0 = __shfl(A.out[0][0], i, 64), f1 = __shfl(A.out[0][1], i, 64),
                        f2 = __shfl(A.out[0][2], i, 64), f3 = __shfl(A.out[0][3], i, 64);
            const float logit = q == 1 ? f0 : (q == 2 ? f1 : f2);
            const float e = expf(q == 0 ? A.o[0][0] : -logit);
            const float sg = 1.0f / (1.0f + e);
            float v = q == 0 ? e : sg;
            if (a.CO != 3 && q != 0) v = v * sigmoidf(f3);
            if (valid) ob[s * ostride] = ok ? v : 0.0f;
        }
        if (more) issue_dirs_of(nx);
    };
    In b0, b1;
    int64_t u = blockIdx.x;
    if (u < total) {
        issue(u, b0);
        issue_dirs_of(b0);
    }
    for (; u < total; u += 2 * (int64_t)gridDim.x) {
        step(u, b0, b1);
        if (u + gridDim.x >= total) break;
        step(u + gridDim.x, b1, b0);
    }
}

// ---- adjoint ----------------------------------------------------------------

// Padded weight-gradient row of one block and weight set: D1 [64][32] | D2
// [16][64] | C1 [64][32] | C2 [64][64] (two colour layers) | CO [16][64].
template <int CL>
struct PadRow {
    static constexpr int D1 = 0, D2 = 2048, C1 = 3072, C2 = 5120;
    static constexpr int CO = C2 + (CL == 2 ? 4096 : 0);
    static constexpr int W = CO + 1024;
};

// Position of packed weight p in the padded row.
__device__ __forceinline__ int padded_index(const MlpArgs &a, int p)
{
    const int C2 = 5120, CO = C2 + (a.CL == 2 ? 4096 : 0);
    if (p < a.off[1]) return p;
    if (p < a.off[2]) return 2048 + (p - a.off[1]);
    if (p < a.off[2] + 64 * a.cin_real) {
        const int e = p - a.off[2], h = e / a.cin_real, c = e - h * a.cin_real;
        return 3072 + h * 32 + (c < 15 ? c + 1 : 16 + (c - 15));
    }
    if (a.CL == 2 && p < a.off[4]) return C2 + (p - a.off[3]);
    return CO + (p - a.off[4]);
}

// Weight gradients sum over samples, so both factors need samples along K,
// while the chain leaves lane (i, q) holding rows 4q..4q+3 of sample i: each
// layer's (dy, x) pair is transposed through LDS before its MFMA.  Two ways
// to hold the sums:
//  - per wavefront (FP32 form): a wavefront stages its own 16 samples and
//    holds the whole of every layer's accumulators; at the end the four
//    wavefronts' sums are added in a fixed order.  The FP32 fragments fill
//    half the LDS, so one block runs per CU and block barriers would only
//    cost.
//  - split across the block (BF16 form): the four wavefronts stage their
//    samples side by side ([row][64 samples], BF16 values) and after one
//    barrier each accumulates a quarter of the layer's 16x16 tiles over all
//    64 samples, so it holds a quarter of the accumulators.  That brings the
//    kernel under 256 registers: two wavefronts per SIMD, which hide each
//    other's latencies.  Two staging buffers alternate, one barrier a layer.

// Tile shape of a layer's weight gradient: TO x TI tiles of 16x16, dy has
// 16 TO rows and x 16 TI rows; `cols` = 16 TI is the row length in PadRow.
template <int M>
struct LayerShape;
template <>
struct LayerShape<M_D1> {
    static constexpr int TO = 4, TI = 2;
};
template <>
struct LayerShape<M_D2> {
    static constexpr int TO = 1, TI = 4;
};
template <>
struct LayerShape<M_C1> {
    static constexpr int TO = 4, TI = 2;
};
template <>
struct LayerShape<M_C2> {
    static constexpr int TO = 4, TI = 4;
};
template <>
struct LayerShape<M_CO> {
    static constexpr int TO = 1, TI = 4;
};

template <int CL, int M>
__device__ constexpr int pad_offset()
{
    typedef PadRow<CL> PR;
    return M == M_D1 ? PR::D1 : M == M_D2 ? PR::D2 : M == M_C1 ? PR::C1 : M == M_C2 ? PR::C2 : PR::CO;
}

template <int N>
__device__ __forceinline__ void zero(f4 (&acc)[N])
{
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
}

template <int PREC, int CL, bool SPLIT>
struct WGrad;

// ---- per wavefront ----
constexpr int kWaveStride = 20;  // floats per staged row (16 samples + pad)
constexpr int kWaveRows = 128;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int PREC, int CL>
struct WGrad<PREC, CL, false> {
    static constexpr int kLdsBytes = 4 * kWaveRows * kWaveStride * (int)sizeof(float);
    static_assert(PadRow<CL>::W * (int)sizeof(float) <= kLdsBytes, "reduction buffer");
    f4 d1[4 * 2], d2[1 * 4], c1[4 * 2], c2[4 * 4], co[1 * 4];   // tile (to, ti) at to TI + ti
    float *R, *st;

    __device__ explicit WGrad(void *lds)
        : R(static_cast<float *>(lds)), st(static_cast<float *>(lds) + (threadIdx.x >> 6) * kWaveRows * kWaveStride)
    {
    }

    template <int M>
    __device__ __forceinline__ auto &acc()
    {
        if constexpr (M == M_D1) return d1;
        else if constexpr (M == M_D2) return d2;
        else if constexpr (M == M_C1) return c1;
        else if constexpr (M == M_C2) return c2;
        else return co;
    }

    __device__ __forceinline__ void zero_all()
    {
        zero(d1);
        zero(d2);
        zero(c1);
        zero(c2);
        zero(co);
    }

    // rows row0 + (0..16T-1) of the wavefront's 16 samples as [row][sample]
    template <int T>
    __device__ __forceinline__ void stage(int row0, const float (&v)[T][4])
    {
        const int lane = lane_id(), i = lane & 15, q = lane >> 4;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) st[(row0 + 16 * t + 4 * q + r) * kWaveStride + i] = v[t][r];
    }

    // acc += dy . x^T over the wavefront's 16 samples
    template <int M>
    __device__ __forceinline__ void layer(const float (&dy)[LayerShape<M>::TO][4],
                                          const float (&x)[LayerShape<M>::TI][4])
    {
        constexpr int TO = LayerShape<M>::TO, TI = LayerShape<M>::TI;
        f4(&a)[TO * TI] = acc<M>();
        stage<TO>(0, dy);
        stage<TI>(16 * TO, x);
        wave_sync();
        const int lane = lane_id(), i = lane & 15, q = lane >> 4;
        f4 av[TO], bv[TI];
#pragma unroll
        for (int to = 0; to < TO; ++to) av[to] = *reinterpret_cast<const f4 *>(st + (16 * to + i) * kWaveStride + 4 * q);
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
            bv[ti] = *reinterpret_cast<const f4 *>(st + (16 * TO + 16 * ti + i) * kWaveStride + 4 * q);
        if constexpr (PREC == P_F32) {
#pragma unroll
            for (int to = 0; to < TO; ++to)
#pragma unroll
                for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        a[to * TI + ti] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(av[to][k], bv[ti][k], a[to * TI + ti], 0, 0, 0);
        } else {
            s4 ab[TO], bb[TI];
#pragma unroll
            for (int to = 0; to < TO; ++to) {
                bf4 t4;
#pragma unroll
                for (int k = 0; k < 4; ++k) t4[k] = (__bf16)av[to][k];
                ab[to] = __builtin_bit_cast(s4, t4);
            }
#pragma unroll
            for (int ti = 0; ti < TI; ++ti) {
                bf4 t4;
#pragma unroll
                for (int k = 0; k < 4; ++k) t4[k] = (__bf16)bv[ti][k];
                bb[ti] = __builtin_bit_cast(s4, t4);
            }
#pragma unroll
            for (int to = 0; to < TO; ++to)
#pragma unroll
                for (int ti = 0; ti < TI; ++ti)
                    a[to * TI + ti] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab[to], bb[ti], a[to * TI + ti], 0, 0, 0);
        }
        wave_sync();
    }

    // one layer's tiles into the row buffer: the first wavefront stores, the
    // others add
    template <int M>
    __device__ __forceinline__ void add_layer(bool first)
    {
        constexpr int TO = LayerShape<M>::TO, TI = LayerShape<M>::TI, cols = 16 * TI;
        const f4(&a)[TO * TI] = acc<M>();
        const int lane = lane_id(), j = lane & 15, q = lane >> 4;
#pragma unroll
        for (int to = 0; to < TO; ++to)
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float *p = R + pad_offset<CL, M>() + (16 * to + 4 * q + r) * cols + 16 * ti + j;
                    *p = first ? a[to * TI + ti][r] : *p + a[to * TI + ti][r];
                }
    }

    // the four wavefronts' sums added in a fixed order, then the padded row
    // out.  Block-uniform: every thread calls it.
    __device__ void flush(float *out)
    {
        const int wv = threadIdx.x >> 6;
        __syncthreads();
        for (int w = 0; w < kBlock / 64; ++w) {
            if (wv == w) {
                add_layer<M_D1>(w == 0);
                add_layer<M_D2>(w == 0);
                add_layer<M_C1>(w == 0);
                if (CL == 2) add_layer<M_C2>(w == 0);
                add_layer<M_CO>(w == 0);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < PadRow<CL>::W / 4; e += kBlock)
            reinterpret_cast<f4 *>(out)[e] = reinterpret_cast<const f4 *>(R)[e];
        __syncthreads();
    }
};

// ---- split across the block ----
template <int PREC>
struct StageT {
    typedef float T;
    static constexpr int stride = 68;   // 64 samples + pad, rows 16-byte aligned
};
template <>
struct StageT<P_BF16> {
    typedef __bf16 T;
    static constexpr int stride = 72;
};
constexpr int kStageRows = 128;         // the largest pair: 64 dy rows + 64 x rows

// A wavefront's tiles of a TO x TI tile layer: e = wv NT + j, all in dy row
// block `to`, x column blocks ti0 + j.
template <int TO, int TI>
struct TileSplit {
    static constexpr int NT = TO * TI / 4;
    static_assert(NT >= 1 && TI % NT == 0, "a wavefront's tiles share one row block");
    __device__ static int to(int wv) { return wv * NT / TI; }
    __device__ static int ti0(int wv) { return wv * NT % TI; }
};

template <int PREC, int CL>
struct WGrad<PREC, CL, true> {
    typedef typename StageT<PREC>::T ST;
    static constexpr int S = StageT<PREC>::stride, kElems = kStageRows * S;
    static constexpr int kLdsBytes = 2 * kElems * (int)sizeof(ST);
    f4 d1[TileSplit<4, 2>::NT], d2[TileSplit<1, 4>::NT], c1[TileSplit<4, 2>::NT], c2[TileSplit<4, 4>::NT],
        co[TileSplit<1, 4>::NT];
    ST *buf;
    int pb;                     // buffer of the next layer (block-uniform)

    __device__ explicit WGrad(void *lds) : buf(static_cast<ST *>(lds)), pb(0) {}

    template <int M>
    __device__ __forceinline__ auto &acc()
    {
        if constexpr (M == M_D1) return d1;
        else if constexpr (M == M_D2) return d2;
        else if constexpr (M == M_C1) return c1;
        else if constexpr (M == M_C2) return c2;
        else return co;
    }

    __device__ __forceinline__ void zero_all()
    {
        zero(d1);
        zero(d2);
        zero(c1);
        zero(c2);
        zero(co);
    }

    // rows row0 + (0..16T-1) of the wavefront's 16 samples into columns 16 wv + i
    template <int T>
    __device__ __forceinline__ void stage(ST *b, int row0, const float (&v)[T][4])
    {
        const int lane = lane_id(), i = lane & 15, q = lane >> 4, col = 16 * (int)(threadIdx.x >> 6) + i;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) b[(row0 + 16 * t + 4 * q + r) * S + col] = (ST)v[t][r];
    }

    // acc[j] += dy[16 to.. ] . x[16 (ti0 + j).. ]^T over the block's 64
    // samples; lane (i, q) supplies samples 16q..16q+15 of row i to both
    // operands
    template <int M>
    __device__ __forceinline__ void layer(const float (&dy)[LayerShape<M>::TO][4],
                                          const float (&x)[LayerShape<M>::TI][4])
    {
        constexpr int TO = LayerShape<M>::TO, TI = LayerShape<M>::TI;
        typedef TileSplit<TO, TI> TS;
        f4(&a)[TS::NT] = acc<M>();
        ST *b = buf + pb * kElems;
        pb ^= 1;
        stage<TO>(b, 0, dy);
        stage<TI>(b, 16 * TO, x);
        __syncthreads();
        const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
        const ST *pa = b + (16 * TS::to(wv) + i) * S + 16 * q;
        const ST *pbx = b + (16 * TO + 16 * TS::ti0(wv) + i) * S + 16 * q;
        if constexpr (PREC == P_F32) {
            f4 av[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) av[h] = *reinterpret_cast<const f4 *>(pa + 4 * h);
#pragma unroll
            for (int j = 0; j < TS::NT; ++j)
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const f4 bv = *reinterpret_cast<const f4 *>(pbx + 16 * j * S + 4 * h);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        a[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[h][k], bv[k], a[j], 0, 0, 0);
                }
        } else {
            bf8 av[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) av[h] = *reinterpret_cast<const bf8 *>(pa + 8 * h);
#pragma unroll
            for (int j = 0; j < TS::NT; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf8 bv = *reinterpret_cast<const bf8 *>(pbx + 16 * j * S + 8 * h);
                    a[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[h], bv, a[j], 0, 0, 0);
                }
        }
    }

    // this wavefront's tiles of a layer into the padded row; the four
    // wavefronts' tiles cover it
    template <int M>
    __device__ __forceinline__ void store_layer(float *out)
    {
        constexpr int TO = LayerShape<M>::TO, TI = LayerShape<M>::TI, cols = 16 * TI;
        typedef TileSplit<TO, TI> TS;
        const f4(&a)[TS::NT] = acc<M>();
        const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
        const int to = TS::to(wv), ti0 = TS::ti0(wv);
        float *o = out + pad_offset<CL, M>();
#pragma unroll
        for (int j = 0; j < TS::NT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) o[(16 * to + 4 * q + r) * cols + 16 * (ti0 + j) + i] = a[j][r];
    }

    __device__ void flush(float *out)
    {
        store_layer<M_D1>(out);
        store_layer<M_D2>(out);
        store_layer<M_C1>(out);
        if constexpr (CL == 2) store_layer<M_C2>(out);
        store_layer<M_CO>(out);
    }
};

template <typename FT>
__device__ __forceinline__ void store_dfeat(float *dfeat, int64_t ld, int64_t s, bool valid, const MlpArgs &a,
                                            const float (&dx)[2][4])
{
    const int q = lane_id() >> 4;
    if (!valid) return;
    if (a.F == 2) {
        float *base = dfeat + ((int64_t)(2 * q) * ld + s) * 2;     // level 8t + 2q + h
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = 16 * t + 4 * q + 2 * h;
                if (p < a.n_feat)
                    *reinterpret_cast<float2 *>(base + (int64_t)(8 * t + h) * ld * 2) =
                        make_float2(dx[t][2 * h], dx[t][2 * h + 1]);
            }
        return;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * t + 4 * q + r;
            if (p < a.n_feat) {
                const int lvl = p / a.F, f = p - lvl * a.F;
                dfeat[((int64_t)lvl * ld + s) * a.F + f] = dx[t][r];
            }
        }
}

template <int PREC, int CL, typename FT, bool LOAD>
__global__ __launch_bounds__(kBlock, PREC == P_BF16 ? 2 : 1) void mlp_bwd_kernel(
    MlpArgs a, const float *__restrict__ w, const FT *__restrict__ feat, int64_t feat_ld,
    const float *__restrict__ view, const float *__restrict__ sun, const int32_t *__restrict__ ray_id,
    const int32_t *__restrict__ sidx, int64_t n, const int64_t *__restrict__ n_dev,
    const float *__restrict__ dsigma, const float *__restrict__ drgb, const float *__restrict__ act,
    float *__restrict__ dfeat, float *__restrict__ partial, const typename FragT<PREC>::T *__restrict__ frag)
{
    typedef Layout<PREC, CL> Lt;
    typedef WGrad<PREC, CL, PREC == P_BF16> WG;
    __shared__ __attribute__((aligned(16))) typename Lt::T lds[Lt::ALL];
    __shared__ __attribute__((aligned(16))) unsigned char wg_lds[WG::kLdsBytes];
    __shared__ UnitTable U;
    const int64_t ne = effective_n(n, n_dev);
    setup_units(U, a, ne);
    const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
    WG wg(wg_lds);

    // inputs of the next unit are loaded while the current one is computed
    int64_t g1 = 0, gbase = 0;   // end of the current group; sample of unit 0 in its numbering
    const int lofs = 16 * wv + i;
    // the index chain (list entry -> sample -> ray) of the next unit is
    // resolved while the current unit is computed
    auto load_idx = [&](int u, BwdIdx &in) {
        in.s = gbase + 64 * (int64_t)u + lofs;
        in.in_range = in.s < g1;
        in.si = in.in_range ? (sidx ? sidx[in.s] : in.s) : 0;
        in.ray = in.in_range ? ray_id[in.si] : 0;
    };
    auto load_data = [&](const BwdIdx &ix, BwdIn &in) {
        in.valid = ix.in_range && ix.ray >= 0 && ix.ray < a.R;    // a bad ray id drops the sample
        if (ix.in_range && !in.valid && q == 0 && a.err) atomicOr(a.err, (unsigned)SNAKE_DEVERR_RAY_ID);
        const int ray = in.valid ? ix.ray : 0;
        load_features(feat, feat_ld, ix.si, in.valid, a, in.x);
        load_dirs(view, sun, ray, in.valid, a, in.dirs);
        in.dsig = in.dr[0] = in.dr[1] = in.dr[2] = 0.0f;
        if (q == 0 && in.valid) {
            in.dsig = dsigma[ix.si];
#pragma unroll
            for (int c = 0; c < 3; ++c) in.dr[c] = drgb[3 * ix.si + c];
        }
    };
    const int G = (int)gridDim.x;
    for (int k = 0; k <= a.K; ++k) {                          // block-uniform
        // this block's units of group k: u = blockIdx.x (mod G) in [ub[k], ub[k+1])
        const int ua = (int)U.ub[k], ue = (int)U.ub[k + 1];
        int u = ua + (((int)blockIdx.x - ua) % G + G) % G;
        if (u >= ue) continue;
        g1 = U.ts[k + 1];
        gbase = U.ts[k] - 64 * (int64_t)ua;
        if (k == a.K) {                                       // invalid tile id: dropped
            const float zx[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
            for (; u < ue; u += G) {
                const int64_t s = gbase + 64 * (int64_t)u + lofs;
                store_dfeat<FT>(dfeat, n, s, s < g1, a, zx);
            }
            continue;
        }
        {
            // tile k's fragments, prepared once by mlp_frag_kernel, into LDS
            constexpr int n16 = Lt::ALL * (int)sizeof(typename Lt::T) / 16;
            const uint4 *src = reinterpret_cast<const uint4 *>(frag + (int64_t)k * Lt::ALL);
            uint4 *dst = reinterpret_cast<uint4 *>(lds);
            __syncthreads();
            for (int e = threadIdx.x; e < n16; e += kBlock) dst[e] = src[e];
            __syncthreads();
        }
        wg.zero_all();
        BwdIdx ix;
        load_idx(u, ix);
        for (; u < ue; u += G) {
            BwdIn cur;
            load_data(ix, cur);
            const int64_t s = ix.s, si = ix.si;
            const bool in_range = ix.in_range, valid = cur.valid;
            if (u + G < ue) load_idx(u + G, ix);
            Acts<PREC, CL> A;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r) A.x[h][r] = cur.x[h][r];
#pragma unroll
            for (int r = 0; r < 4; ++r) A.cin[1][r] = cur.dirs[r];
            if constexpr (LOAD) {
                if (valid) {
                    load_acts<PREC, CL>(act + si * ActLayout<CL>::W, A);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        A.o[0][r] = A.cin[0][r] = A.out[0][r] = 0.0f;
#pragma unroll
                        for (int t = 0; t < 4; ++t) A.h1[t][r] = A.g1[t][r] = A.g2[t][r] = 0.0f;
                    }
                }
            } else {
                forward_tile<PREC, CL>(lds, A);
            }

            // output activation adjoint (rows 0..3 live in lane group 0)
            float dout[1][4] = {{0.f, 0.f, 0.f, 0.f}};
            const float dsig = cur.dsig;
            if (q == 0 && valid) {
                const float *dr = cur.dr;
                if (a.CO == 3) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float y = sigmoidf(A.out[0][c]);
                        dout[0][c] = dr[c] * y * (1.0f - y);
                    }
                } else {
                    const float vis = sigmoidf(A.out[0][3]);
                    float dvis = 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float alb = sigmoidf(A.out[0][c]);
                        dout[0][c] = dr[c] * vis * alb * (1.0f - alb);
                        dvis += dr[c] * alb;
                    }
                    dout[0][3] = dvis * vis * (1.0f - vis);
                }
            }
            // adjoint chain; each layer's weight gradient as soon as both of
            // its factors are known
            float dg2[4][4], dg1[4][4], dob[1][4], dh1[4][4], dx[2][4];
            if constexpr (CL == 2) {
                apply<PREC, 64, 16>(lds + Lt::COT, dout, dg2);
                relu_mask(dg2, A.g2);
                wg.template layer<M_CO>(dout, A.g2);
                apply<PREC, 64, 64>(lds + Lt::C2T, dg2, dg1);
                relu_mask(dg1, A.g1);
                wg.template layer<M_C2>(dg2, A.g1);
            } else {
                apply<PREC, 64, 16>(lds + Lt::COT, dout, dg1);
                relu_mask(dg1, A.g1);
                wg.template layer<M_CO>(dout, A.g1);
            }
            apply<PREC, 16, 64>(lds + Lt::C1T, dg1, dob);
            if (q == 0) dob[0][0] = dsig * expf(A.o[0][0]);   // sigma = exp(o_0)
            wg.template layer<M_C1>(dg1, A.cin);
            apply<PREC, 64, 16>(lds + Lt::D2T, dob, dh1);
            relu_mask(dh1, A.h1);
            wg.template layer<M_D2>(dob, A.h1);
            apply<PREC, 32, 64>(lds + Lt::D1T, dh1, dx);
            store_dfeat<FT>(dfeat, n, s, in_range, a, dx);       // dropped samples store zeros
            wg.template layer<M_D1>(dh1, A.x);
        }
        wg.flush(partial + ((int64_t)blockIdx.x * a.K + k) * PadRow<CL>::W);
    }
}

// The adjoint for F == 2 with recomputed activations, software-pipelined
// like the forward: the index list entry of unit u + 2 grid, the ray id,
// features and output gradients of unit u + grid, and (after the current
// unit) the directions of unit u + grid are in flight while unit u is
// computed.  Loads go to valid addresses without branches, into two
// alternating buffers, and nothing reads them before the layer that needs
// them.  Results are those of mlp_bwd_kernel bit for bit.
template <int PREC, int CL, typename FT>
__global__ __launch_bounds__(kBlock, PREC == P_BF16 ? 2 : 1) void mlp_bwd_pipe_kernel(
    MlpArgs a, const float *__restrict__ w, const FT *__restrict__ feat, int64_t feat_ld,
    const float *__restrict__ view, const float *__restrict__ sun, const int32_t *__restrict__ ray_id,
    const int32_t *__restrict__ sidx, int64_t n, const int64_t *__restrict__ n_dev,
    const float *__restrict__ dsigma, const float *__restrict__ drgb, float *__restrict__ dfeat,
    float *__restrict__ partial, const typename FragT<PREC>::T *__restrict__ frag)
{
    typedef Layout<PREC, CL> Lt;
    typedef WGrad<PREC, CL, PREC == P_BF16> WG;
    __shared__ __attribute__((aligned(16))) typename Lt::T lds[Lt::ALL];
    __shared__ __attribute__((aligned(16))) unsigned char wg_lds[WG::kLdsBytes];
    __shared__ UnitTable U;
    const int64_t ne = effective_n(n, n_dev);
    setup_units(U, a, ne);
    const int lane = lane_id(), i = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
    WG wg(wg_lds);
    const int lofs = 16 * wv + i;

    struct D {
        int64_t s;
        bool in_range;
        int32_t ray;
        uint32_t use, dmask;
        RawFeat<FT> raw;
        float dsig, dr[3], dirs[4];
    };
    int64_t g0 = 0, g1 = 0, gbase = 0;   // group's first entry and end; entry of unit 0 in its numbering
    auto si_of = [&](int uu) -> int64_t {
        const int64_t s = gbase + 64 * (int64_t)uu + lofs;
        const int64_t sc = s < g1 ? s : g0;                  // an entry that exists
        return sidx ? (int64_t)sidx[sc] : sc;
    };
    auto issue_data = [&](int uu, int64_t si, D &d) {
        d.s = gbase + 64 * (int64_t)uu + lofs;
        d.in_range = d.s < g1;
        d.ray = ray_id[si];
        issue_features<FT>(feat, feat_ld, si, d.in_range, a, d.raw, d.use);
        d.dsig = dsigma[si];
#pragma unroll
        for (int c = 0; c < 3; ++c) d.dr[c] = drgb[3 * si + c];
    };
    auto issue_dirs_of = [&](D &d) {
        const bool ok = d.in_range && d.ray >= 0 && d.ray < a.R;
        issue_dirs(view, sun, ok ? d.ray : 0, a, d.dirs, d.dmask);
    };
    auto compute = [&](const D &x) {
        const bool valid = x.in_range && x.ray >= 0 && x.ray < a.R;   // a bad ray id drops the sample
        if (x.in_range && !valid && q == 0 && a.err) atomicOr(a.err, (unsigned)SNAKE_DEVERR_RAY_ID);
        Acts<PREC, CL> A;
        __builtin_amdgcn_sched_barrier(0);
        take_features<FT>(x.raw, x.use, valid, A.x);
        apply<PREC, 64, 32>(lds + Lt::D1, A.x, A.h1);
        relu(A.h1);
        apply<PREC, 16, 64>(lds + Lt::D2, A.h1, A.o);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            A.cin[0][r] = A.o[0][r];
            A.cin[1][r] = valid && ((x.dmask >> r) & 1u) ? x.dirs[r] : 0.0f;
        }
        apply<PREC, 64, 32>(lds + Lt::C1, A.cin, A.g1);
        relu(A.g1);
        if constexpr (CL == 2) {
            apply<PREC, 64, 64>(lds + Lt::C2, A.g1, A.g2);
            relu(A.g2);
            apply<PREC, 16, 64>(lds + Lt::CO, A.g2, A.out);
        } else {
            apply<PREC, 16, 64>(lds + Lt::CO, A.g1, A.out);
        }
        // output activation adjoint (rows 0..3 live in lane group 0)
        float dout[1][4] = {{0.f, 0.f, 0.f, 0.f}};
        const bool lead = q == 0 && valid;
        const float dsig = lead ? x.dsig : 0.0f;
        if (lead) {
            if (a.CO == 3) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float y = sigmoidf(A.out[0][c]);
                    dout[0][c] = x.dr[c] * y * (1.0f - y);
                }
            } else {
                const float vis = sigmoidf(A.out[0][3]);
                float dvis = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float alb = sigmoidf(A.out[0][c]);
                    dout[0][c] = x.dr[c] * vis * alb * (1.0f - alb);
                    dvis += x.dr[c] * alb;
                }
                dout[0][3] = dvis * vis * (1.0f - vis);
            }
        }
        float dg2[4][4], dg1[4][4], dob[1][4], dh1[4][4], dx[2][4];
        if constexpr (CL == 2) {
            apply<PREC, 64, 16>(lds + Lt::COT, dout, dg2);
            relu_mask(dg2, A.g2);
            wg.template layer<M_CO>(dout, A.g2);
            apply<PREC, 64, 64>(lds + Lt::C2T, dg2, dg1);
            relu_mask(dg1, A.g1);
            wg.template layer<M_C2>(dg2, A.g1);
        } else {
            apply<PREC, 64, 16>(lds + Lt::COT, dout, dg1);
            relu_mask(dg1, A.g1);
            wg.template layer<M_CO>(dout, A.g1);
        }
        apply<PREC, 16, 64>(lds + Lt::C1T, dg1, dob);
        if (q == 0) dob[0][0] = dsig * expf(A.o[0][0]);   // sigma = exp(o_0)
        wg.template layer<M_C1>(dg1, A.cin);
        apply<PREC, 64, 16>(lds + Lt::D2T, dob, dh1);
        relu_mask(dh1, A.h1);
        wg.template layer<M_D2>(dob, A.h1);
        apply<PREC, 32, 64>(lds + Lt::D1T, dh1, dx);
        store_dfeat<FT>(dfeat, n, x.s, x.in_range, a, dx);   // dropped samples store zeros
        wg.template layer<M_D1>(dh1, A.x);
    };

    const int G = (int)gridDim.x;
    for (int k = 0; k <= a.K; ++k) {                          // block-uniform
        // this block's units of group k: u = blockIdx.x (mod G) in [ub[k], ub[k+1])
        const int ua = (int)U.ub[k], ue = (int)U.ub[k + 1];
        int u = ua + (((int)blockIdx.x - ua) % G + G) % G;
        if (u >= ue) continue;
        g0 = U.ts[k];
        g1 = U.ts[k + 1];
        gbase = U.ts[k] - 64 * (int64_t)ua;
        if (k == a.K) {                                       // invalid tile id: dropped
            const float zx[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
            for (; u < ue; u += G) {
                const int64_t s = gbase + 64 * (int64_t)u + lofs;
                store_dfeat<FT>(dfeat, n, s, s < g1, a, zx);
            }
            continue;
        }
        {
            // tile k's fragments, prepared once by mlp_frag_kernel, into LDS
            constexpr int n16 = Lt::ALL * (int)sizeof(typename Lt::T) / 16;
            const uint4 *src = reinterpret_cast<const uint4 *>(frag + (int64_t)k * Lt::ALL);
            uint4 *dst = reinterpret_cast<uint4 *>(lds);
            __syncthreads();
            for (int e = threadIdx.x; e < n16; e += kBlock) dst[e] = src[e];
            __syncthreads();
        }
        wg.zero_all();
        D X, Y;
        int64_t si_nx = si_of(u);
        issue_data(u, si_nx, X);
        if (u + G < ue) si_nx = si_of(u + G);
        issue_dirs_of(X);
        // one unit: compute `cur`, with unit uu + G loading into `nxt`
        auto step = [&](int uu, D &cur, D &nxt) {
            const bool more = uu + G < ue;
            if (more) issue_data(uu + G, si_nx, nxt);
            if (uu + 2 * G < ue) si_nx = si_of(uu + 2 * G);
            compute(cur);
            if (more) issue_dirs_of(nxt);
        };
        for (; u < ue; u += 2 * G) {
            step(u, X, Y);
            if (u + G >= ue) break;
            step(u + G, Y, X);
        }
        wg.flush(partial + ((int64_t)blockIdx.x * a.K + k) * PadRow<CL>::W);
    }
}

// Matrix-core fragments (forward and transposed) of weight set blockIdx.x,
// in the LDS layout of the adjoint kernel.
template <int PREC, int CL>
__global__ __launch_bounds__(kBlock) void mlp_frag_kernel(MlpArgs a, const float *__restrict__ w,
                                                          typename FragT<PREC>::T *__restrict__ frag)
{
    typedef Layout<PREC, CL> Lt;
    typename Lt::T *dst = frag + (int64_t)blockIdx.x * Lt::ALL;
    const float *wd, *wc;
    tile_weights(a, w, blockIdx.x, wd, wc);
    build_forward<PREC, CL>(dst, wd, wc, a);
    build_frag<PREC, 64, 16>(dst + Lt::COT, wc, a, M_CO, true);
    if (CL == 2) build_frag<PREC, 64, 64>(dst + Lt::C2T, wc, a, M_C2, true);
    build_frag<PREC, 16, 64>(dst + Lt::C1T, wc, a, M_C1, true);
    build_frag<PREC, 64, 16>(dst + Lt::D2T, wd, a, M_D2, true);
    build_frag<PREC, 32, 64>(dst + Lt::D1T, wd, a, M_D1, true);
}

// dW += the sums, over the blocks that processed units of each weight set, of
// their padded rows.  Which blocks those are follows from the same unit table
// the adjoint used (block b takes units u = b mod grid).  Per-tile sets:
// dW[k][p] sums set k's rows.  Shared colour net: dW[k][p] for the density
// part of set k, then one colour part summed over all sets.  A block handles
// 64 parameters (one per lane); its kRedGroups wavefronts each sum every
// kRedGroups-th block row (sets in order, blocks ascending), and the groups'
// sums are added in group order: a fixed order, so the result is the same
// every run.
constexpr int kRedGroups = 16;

__global__ __launch_bounds__(64 * kRedGroups) void reduce_partials_kernel(MlpArgs a, const float *__restrict__ partial,
                                                                          int nb, int W, int64_t n,
                                                                          const int64_t *__restrict__ n_dev,
                                                                          float *__restrict__ dW)
{
    __shared__ UnitTable U;
    __shared__ float part[kRedGroups][64];
    setup_units(U, a, effective_n(n, n_dev));
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int Pc = a.P - a.Pd;
    const int64_t total = a.shared_colour ? (int64_t)a.K * a.Pd + Pc : (int64_t)a.K * a.P;
    for (int64_t e0 = (int64_t)blockIdx.x * 64; e0 < total; e0 += (int64_t)gridDim.x * 64) {   // block-uniform
        const int64_t e = e0 + lane;
        float s = 0.0f;
        if (e < total) {
            int k0, k1, p;
            if (!a.shared_colour) {
                k0 = (int)(e / a.P);
                p = (int)(e - (int64_t)k0 * a.P);
                k1 = k0 + 1;
            } else if (e < (int64_t)a.K * a.Pd) {
                k0 = (int)(e / a.Pd);
                p = (int)(e - (int64_t)k0 * a.Pd);
                k1 = k0 + 1;
            } else {
                k0 = 0;
                k1 = a.K;
                p = a.Pd + (int)(e - (int64_t)a.K * a.Pd);
            }
            const int pi = padded_index(a, p);
            for (int k = k0; k < k1; ++k) {
                const int ua = (int)U.ub[k], ue = (int)U.ub[k + 1];
                const float *src = partial + (int64_t)k * W + pi;
                for (int b = grp; b < nb; b += kRedGroups) {
                    const int u = ua + ((b - ua) % nb + nb) % nb;   // block b's first unit of set k
                    if (u < ue) s += src[(int64_t)b * a.K * W];
                }
            }
        }
        part[grp][lane] = s;
        __syncthreads();
        if (grp == 0 && e < total) {
            float t = 0.0f;
#pragma unroll
            for (int g = 0; g < kRedGroups; ++g) t += part[g][lane];
            dW[e] += t;
        }
        __syncthreads();
    }
}

int make_args(const snake_mlp_desc *m, int64_t R, MlpArgs &a, const char *fn, int K = 1,
              const int64_t *tile_start = nullptr)
{
    SNAKE_REQUIRE(K >= 1 && K <= kMaxMlpTiles, SNAKE_ERR_INVALID_ARG, "%s: K = %d not in [1, %d]", fn, K,
                  kMaxMlpTiles);
    SNAKE_REQUIRE(K == 1 || tile_start != nullptr, SNAKE_ERR_NULL, "%s: tile_start is NULL with K = %d", fn, K);
    a.K = K;
    a.tile_start = tile_start;
    SNAKE_REQUIRE(m != nullptr, SNAKE_ERR_NULL, "%s: MLP descriptor is NULL", fn);
    SNAKE_REQUIRE(m->n_levels >= 1 && (m->n_features == 1 || m->n_features == 2 || m->n_features == 4),
                  SNAKE_ERR_INVALID_ARG, "%s: bad encoding shape L=%d F=%d", fn, m->n_levels, m->n_features);
    SNAKE_REQUIRE(m->n_levels * m->n_features <= 32, SNAKE_ERR_INVALID_ARG, "%s: L*F = %d > 32", fn,
                  m->n_levels * m->n_features);
    SNAKE_REQUIRE(m->n_dir == 3 || m->n_dir == 6, SNAKE_ERR_INVALID_ARG, "%s: n_dir = %d not 3 or 6", fn,
                  m->n_dir);
    SNAKE_REQUIRE(m->colour_layers == 1 || m->colour_layers == 2, SNAKE_ERR_UNSUPPORTED,
                  "%s: colour_layers = %d not 1 or 2", fn, m->colour_layers);
    SNAKE_REQUIRE(m->colour_out == 3 || m->colour_out == 4, SNAKE_ERR_INVALID_ARG,
                  "%s: colour_out = %d not 3 or 4", fn, m->colour_out);
    SNAKE_REQUIRE(m->precision == SNAKE_F32 || m->precision == SNAKE_BF16, SNAKE_ERR_INVALID_ARG,
                  "%s: bad precision %d", fn, m->precision);
    SNAKE_REQUIRE(m->feat_dtype == SNAKE_F32 || m->feat_dtype == SNAKE_BF16, SNAKE_ERR_INVALID_ARG,
                  "%s: bad feat_dtype %d", fn, m->feat_dtype);
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "%s: R < 0", fn);
    a.R = R;
    a.err = nullptr;
    a.L = m->n_levels;
    a.F = m->n_features;
    a.n_feat = a.L * a.F;
    a.n_dir = m->n_dir;
    a.CL = m->colour_layers;
    a.CO = m->colour_out;
    a.cin_real = 15 + a.n_dir;
    int64_t o = 0;
    a.off[0] = o;
    o += 64 * 32;
    a.off[1] = o;
    o += 16 * 64;
    a.off[2] = o;
    o += 64 * a.cin_real;
    a.off[3] = o;
    if (a.CL == 2) o += 64 * 64;
    a.off[4] = o;
    o += a.CO * 64;
    a.P = o;
    a.Pd = a.off[2];
    SNAKE_REQUIRE(m->shared_colour == 0 || m->shared_colour == 1, SNAKE_ERR_INVALID_ARG,
                  "%s: shared_colour = %d not 0 or 1", fn, m->shared_colour);
    a.shared_colour = m->shared_colour;
    return SNAKE_OK;
}

// Adjoint workspace: per-block partial rows [blocks][K][P] float, then the
// K weight sets' fragments (FP32 size, the larger of the two forms).
size_t partial_bytes(const MlpArgs &a)
{
    const size_t W = a.CL == 2 ? PadRow<2>::W : PadRow<1>::W;
    return ((size_t)kMaxBwdBlocks * (size_t)a.K * W * sizeof(float) + 255) / 256 * 256;
}

size_t bwd_ws_bytes(const MlpArgs &a)
{
    const size_t frag = a.CL == 2 ? (size_t)Layout<P_F32, 2>::ALL : (size_t)Layout<P_F32, 1>::ALL;
    return partial_bytes(a) + (size_t)a.K * frag * sizeof(float);
}

template <int PREC, int CL, typename FT>
void launch_fwd(const MlpArgs &a, const float *w, const void *feat, const float *view, const float *sun,
                const int32_t *ray_id, const int32_t *sidx, int64_t n, const int64_t *n_dev, float *sigma,
                float *rgb, float *act, hipStream_t st)
{
    const unsigned grid = grid_for(((n + 63) / 64 + a.K) * kBlock, kBlock, tune(SNAKE_TUNE_MLP_FWD_BLOCKS_PER_CU));
    if (a.F == 2 && sidx == nullptr) {
        if (act)
            mlp_fwd_pipe_kernel<PREC, CL, FT, true><<<grid, kBlock, 0, st>>>(
                a, w, static_cast<const FT *>(feat), view, sun, ray_id, n, n_dev, sigma, rgb, act);
        else
            mlp_fwd_pipe_kernel<PREC, CL, FT, false><<<grid, kBlock, 0, st>>>(
                a, w, static_cast<const FT *>(feat), view, sun, ray_id, n, n_dev, sigma, rgb, act);
        return;
    }
    if (act)
        mlp_fwd_kernel<PREC, CL, FT, true><<<grid, kBlock, 0, st>>>(a, w, static_cast<const FT *>(feat), view, sun,
                                                                    ray_id, sidx, n, n_dev, sigma, rgb, act);
    else
        mlp_fwd_kernel<PREC, CL, FT, false><<<grid, kBlock, 0, st>>>(a, w, static_cast<const FT *>(feat), view, sun,
                                                                     ray_id, sidx, n, n_dev, sigma, rgb, act);
}

template <int PREC, int CL, typename FT>
void launch_bwd_pipe(const MlpArgs &a, unsigned grid, const float *w, const void *feat, int64_t feat_ld,
                     const float *view, const float *sun, const int32_t *ray_id, const int32_t *sidx, int64_t n,
                     const int64_t *n_dev, const float *dsigma, const float *drgb, float *dfeat, float *partial,
                     const void *frag, hipStream_t st)
{
    if constexpr (PREC == P_BF16 && !kBwd16Unit) {
        // compiled in mlp_bwd16.hip; launch_bwd calls launch_bwd_pipe_bf16
    } else {
        mlp_bwd_pipe_kernel<PREC, CL, FT><<<grid, kBlock, 0, st>>>(
            a, w, static_cast<const FT *>(feat), feat_ld, view, sun, ray_id, sidx, n, n_dev, dsigma, drgb, dfeat,
            partial, static_cast<const typename FragT<PREC>::T *>(frag));
    }
}

template <int PREC, int CL, typename FT>
void launch_bwd(const MlpArgs &a, const float *w, const void *feat, int64_t feat_ld, const float *view,
                const float *sun, const int32_t *ray_id, const int32_t *sidx, int64_t n, const int64_t *n_dev,
                const float *dsigma, const float *drgb, const float *act, float *dW, float *dfeat, float *partial,
                hipStream_t st)
{
    const int per_cu = tune(SNAKE_TUNE_MLP_BWD_BLOCKS_PER_CU);
    unsigned grid = grid_for(((n + 63) / 64 + a.K) * kBlock, kBlock, per_cu ? per_cu : (PREC == P_BF16 ? 2 : 1));
    if (grid > (unsigned)kMaxBwdBlocks) grid = kMaxBwdBlocks;
    typedef typename FragT<PREC>::T FragEl;
    FragEl *frag = reinterpret_cast<FragEl *>(reinterpret_cast<char *>(partial) + partial_bytes(a));
    mlp_frag_kernel<PREC, CL><<<a.K, kBlock, 0, st>>>(a, w, frag);
    if (!act && a.F == 2 && PREC == P_BF16)
        launch_bwd_pipe_bf16(a, CL, std::is_same<FT, __hip_bfloat16>::value, grid, w, feat, feat_ld, view, sun, ray_id,
                             sidx, n, n_dev, dsigma, drgb, dfeat, partial, frag, st);
    else if (!act && a.F == 2)
        launch_bwd_pipe<PREC, CL, FT>(a, grid, w, feat, feat_ld, view, sun, ray_id, sidx, n, n_dev, dsigma, drgb,
                                      dfeat, partial, frag, st);
    else if (act)
        mlp_bwd_kernel<PREC, CL, FT, true><<<grid, kBlock, 0, st>>>(a, w, static_cast<const FT *>(feat), feat_ld, view,
                                                                    sun, ray_id, sidx, n, n_dev, dsigma, drgb, act,
                                                                    dfeat, partial, frag);
    else
        mlp_bwd_kernel<PREC, CL, FT, false><<<grid, kBlock, 0, st>>>(a, w, static_cast<const FT *>(feat), feat_ld,
                                                                     view, sun, ray_id, sidx, n, n_dev, dsigma, drgb,
                                                                     act, dfeat, partial, frag);
    const int64_t kp = a.shared_colour ? (int64_t)a.K * a.Pd + (a.P - a.Pd) : (int64_t)a.K * a.P;
    reduce_partials_kernel<<<(unsigned)((kp + 63) / 64), 64 * kRedGroups, 0, st>>>(a, partial, (int)grid,
                                                                                    PadRow<CL>::W, n, n_dev, dW);
}

}  // namespace

#ifdef SNAKE_MLP_BWD16
void launch_bwd_pipe_bf16(const MlpArgs &a, int cl, bool feat_bf16, unsigned grid, const float *w, const void *feat,
                          int64_t feat_ld, const float *view, const float *sun, const int32_t *ray_id,
                          const int32_t *sidx, int64_t n, const int64_t *n_dev, const float *dsigma,
                          const float *drgb, float *dfeat, float *partial, const void *frag, hipStream_t st)
{
#define SNAKE_BWD16(C, FT)                                                                                     \
    launch_bwd_pipe<P_BF16, C, FT>(a, grid, w, feat, feat_ld, view, sun, ray_id, sidx, n, n_dev, dsigma, drgb, \
                                   dfeat, partial, frag, st)
    if (cl == 2) {
        if (feat_bf16) SNAKE_BWD16(2, __hip_bfloat16); else SNAKE_BWD16(2, float);
    } else {
        if (feat_bf16) SNAKE_BWD16(1, __hip_bfloat16); else SNAKE_BWD16(1, float);
    }
#undef SNAKE_BWD16
}
#endif
}  // namespace snake

#ifndef SNAKE_MLP_BWD16
using namespace snake;

extern "C" {

int64_t snake_mlp_param_count(const snake_mlp_desc *m)
{
    MlpArgs a;
    if (make_args(m, 0, a, __func__)) return -1;
    return a.P;
}

int64_t snake_mlp_weight_count(const snake_mlp_desc *m, int32_t K)
{
    MlpArgs a;
    if (K < 1 || K > kMaxMlpTiles || make_args(m, 0, a, __func__)) return -1;
    return a.shared_colour ? (int64_t)K * a.Pd + (a.P - a.Pd) : (int64_t)K * a.P;
}

int32_t snake_mlp_act_width(const snake_mlp_desc *m)
{
    MlpArgs a;
    if (make_args(m, 0, a, __func__)) return -1;
    return a.CL == 2 ? ActLayout<2>::W : ActLayout<1>::W;
}

size_t snake_mlp_bwd_workspace_bytes(const snake_mlp_desc *m, int32_t K)
{
    MlpArgs a;
    if (K < 1 || K > kMaxMlpTiles || make_args(m, 0, a, __func__, K, K > 1 ? &kNoTable : nullptr)) return 0;
    return bwd_ws_bytes(a);
}

int snake_mlp_fwd(const snake_mlp_desc *m, int32_t K, const float *weights, const int64_t *tile_start,
                  const void *feat, const float *view, const float *sun, const int32_t *ray_id, int32_t R,
                  const int32_t *sample_idx, int64_t n, const int64_t *n_dev, float *sigma, float *rgb,
                  float *act, snake_stream_t stream)
{
    MlpArgs a;
    int rc = make_args(m, R, a, __func__, K, tile_start);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_mlp_fwd: n < 0");
    if (n == 0) return SNAKE_OK;
    SNAKE_NOT_NULL(weights);
    SNAKE_NOT_NULL(feat);
    SNAKE_NOT_NULL(view);
    SNAKE_NOT_NULL(ray_id);
    SNAKE_NOT_NULL(sigma);
    SNAKE_NOT_NULL(rgb);
    SNAKE_REQUIRE(a.n_dir == 3 || sun != nullptr, SNAKE_ERR_NULL, "snake_mlp_fwd: sun is NULL with n_dir = 6");
    if (a.F == 2) SNAKE_ALIGNED(feat, m->feat_dtype == SNAKE_BF16 ? 4 : 8);
    SNAKE_ALIGNED(act, 16);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    a.err = device_error_word();
    const bool bf = m->precision == SNAKE_BF16, fb = m->feat_dtype == SNAKE_BF16;
#define SNAKE_MLP_FWD(P, C)                                                                                  \
    if (fb)                                                                                                  \
        launch_fwd<P, C, __hip_bfloat16>(a, weights, feat, view, sun, ray_id, sample_idx, n, n_dev, sigma, rgb, \
                                         act, st);                                                           \
    else                                                                                                     \
        launch_fwd<P, C, float>(a, weights, feat, view, sun, ray_id, sample_idx, n, n_dev, sigma, rgb, act, st)
    if (bf) {
        if (a.CL == 2) {
            SNAKE_MLP_FWD(P_BF16, 2);
        } else {
            SNAKE_MLP_FWD(P_BF16, 1);
        }
    } else {
        if (a.CL == 2) {
            SNAKE_MLP_FWD(P_F32, 2);
        } else {
            SNAKE_MLP_FWD(P_F32, 1);
        }
    }
#undef SNAKE_MLP_FWD
    return launch_status(__func__);
}

int snake_mlp_bwd(const snake_mlp_desc *m, int32_t K, const float *weights, const int64_t *tile_start,
                  const void *feat, int64_t feat_ld, const float *view, const float *sun, const int32_t *ray_id,
                  int32_t R,
                  const int32_t *sample_idx, int64_t n, const int64_t *n_dev, const float *dsigma,
                  const float *drgb, const float *act, float *dW, float *dfeat, void *workspace,
                  size_t workspace_bytes, snake_stream_t stream)
{
    MlpArgs a;
    int rc = make_args(m, R, a, __func__, K, tile_start);
    if (rc) return rc;
    SNAKE_REQUIRE(n >= 0, SNAKE_ERR_INVALID_ARG, "snake_mlp_bwd: n < 0");
    if (n == 0) return SNAKE_OK;
    SNAKE_REQUIRE(sample_idx != nullptr || feat_ld >= n, SNAKE_ERR_INVALID_ARG,
                  "snake_mlp_bwd: feat_ld = %lld < n = %lld", (long long)feat_ld, (long long)n);
    SNAKE_NOT_NULL(weights);
    SNAKE_NOT_NULL(feat);
    SNAKE_NOT_NULL(view);
    SNAKE_NOT_NULL(ray_id);
    SNAKE_NOT_NULL(dsigma);
    SNAKE_NOT_NULL(drgb);
    SNAKE_NOT_NULL(dW);
    SNAKE_NOT_NULL(dfeat);
    SNAKE_REQUIRE(a.n_dir == 3 || sun != nullptr, SNAKE_ERR_NULL, "snake_mlp_bwd: sun is NULL with n_dir = 6");
    if (a.F == 2) {
        SNAKE_ALIGNED(feat, m->feat_dtype == SNAKE_BF16 ? 4 : 8);
        SNAKE_ALIGNED(dfeat, 8);
    }
    SNAKE_ALIGNED(act, 16);
    const size_t need = bwd_ws_bytes(a);
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= need, SNAKE_ERR_WORKSPACE,
                  "snake_mlp_bwd: workspace needs %zu bytes", need);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    SNAKE_ALIGNED(workspace, 256);
    float *partial = static_cast<float *>(workspace);
    a.err = device_error_word();
    const bool bf = m->precision == SNAKE_BF16, fb = m->feat_dtype == SNAKE_BF16;
#define SNAKE_MLP_BWD(P, C)                                                                                     \
    if (fb)                                                                                                     \
        launch_bwd<P, C, __hip_bfloat16>(a, weights, feat, feat_ld, view, sun, ray_id, sample_idx, n, n_dev,      \
                                         dsigma, drgb, act, dW, dfeat, partial, st);                            \
    else                                                                                                        \
        launch_bwd<P, C, float>(a, weights, feat, feat_ld, view, sun, ray_id, sample_idx, n, n_dev, dsigma, drgb, \
                                act, dW, dfeat, partial, st)
    if (bf) {
        if (a.CL == 2) {
            SNAKE_MLP_BWD(P_BF16, 2);
        } else {
            SNAKE_MLP_BWD(P_BF16, 1);
        }
    } else {
        if (a.CL == 2) {
            SNAKE_MLP_BWD(P_F32, 2);
        } else {
            SNAKE_MLP_BWD(P_F32, 1);
        }
    }
#undef SNAKE_MLP_BWD
    return launch_status(__func__);
}

}  // extern "C"
#endif  // SNAKE_MLP_BWD16
