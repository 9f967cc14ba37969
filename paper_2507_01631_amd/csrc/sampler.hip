// Segmented sampler: per-NeRF-tile near/far, per-segment uniform intervals,
// count -> exclusive scan -> fill packing (Sec. 4.5, Sec. 4.6; tile-local
// [0,1]^3 frame of Sec. 4.1-4.2).
//
// Bit-exactness: every FP64 and FP32 operation below is a single IEEE
// operation at a stated rounding point, so FMA contraction is off for the
// whole file.
#pragma clang fp contract(off)

#include <math.h>

#include <mutex>

#include "common.h"
#include "scan.h"

namespace snake {
namespace {

constexpr int kMaxTiles = 16;

struct Boxes {
    double b[kMaxTiles][6];
    int K;
    int use_band;
    double z_lo, z_hi;
};

// A ray's hit segments in entry order.  Every array is indexed with
// compile-time indices only (unrolled loops and selects), so the list lives
// in registers: an index computed at run time would put it in scratch memory.
template <int KMAX>
struct Segs {
    double tn[KMAX], tf[KMAX];
    int tile[KMAX];
    int n[KMAX];
    int ns;
};

// FP64 slab test; hit iff t_far > t_near after clamping t_near at 0.  An
// axis-parallel component is inside when lo <= o < hi.
__device__ __forceinline__ bool slab(const double o[3], const double d[3], const double lo[3],
                                     const double hi[3], double &tn, double &tf)
{
    double t_near = -INFINITY, t_far = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] >= hi[a]) return false;
            continue;
        }
        double u = (lo[a] - o[a]) / d[a];
        double v = (hi[a] - o[a]) / d[a];
        double mn = u < v ? u : v;
        double mx = u < v ? v : u;
        t_near = mn > t_near ? mn : t_near;
        t_far = mx < t_far ? mx : t_far;
    }
    t_near = t_near < 0.0 ? 0.0 : t_near;
    if (!(t_far > t_near)) return false;
    tn = t_near;
    tf = t_far;
    return true;
}

// Hit segments of one ray in entry order (ties in the entry point by tile
// index) with their sample counts (sum S_r when S_r > 0).
__device__ __forceinline__ double read_lane(double v, int k)
{
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(w.x, k), __builtin_amdgcn_readlane(w.y, k)));
}

// Box k of the list, clipped to the altitude band when one is set.
template <int KMAX>
__device__ __forceinline__ void box_of(const Boxes &bx, int k, double lo[3], double hi[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = bx.b[0][a];
        hi[a] = bx.b[0][3 + a];
    }
#pragma unroll
    for (int t = 1; t < KMAX; ++t)
        if (k == t) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = bx.b[t][a];
                hi[a] = bx.b[t][3 + a];
            }
        }
    if (bx.use_band) {
        lo[2] = bx.z_lo > lo[2] ? bx.z_lo : lo[2];
        hi[2] = bx.z_hi < hi[2] ? bx.z_hi : hi[2];
    }
}

// Wave = true: called by a whole wavefront for one ray (every lane active,
// the same o and d); lane k tests box k and the others read its result.
template <int KMAX, bool Wave = false>
__device__ __forceinline__ void ray_segments(const double o[3], const double d[3], const Boxes &bx, int S_r,
                                             Segs<KMAX> &sg)
{
    double tn[KMAX], tf[KMAX];
    bool hit[KMAX];
    if constexpr (Wave && KMAX > 1) {
        const int lane = lane_id();
        double mtn = 0.0, mtf = 0.0;
        bool mhit = false;
        if (lane < bx.K) {
            double lo[3], hi[3];
            box_of<KMAX>(bx, lane, lo, hi);
            mhit = slab(o, d, lo, hi, mtn, mtf);
        }
        const unsigned long long hits = __ballot(mhit);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            hit[k] = (hits >> k) & 1ull;
            tn[k] = read_lane(mtn, k);
            tf[k] = read_lane(mtf, k);
        }
    } else {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            hit[k] = false;
            tn[k] = tf[k] = 0.0;
            if (k < bx.K) {
                double lo[3], hi[3];
                box_of<KMAX>(bx, k, lo, hi);
                hit[k] = slab(o, d, lo, hi, tn[k], tf[k]);
            }
        }
    }
    // position of each hit box in (entry point, tile) order
    int rank[KMAX];
    int ns = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        rank[k] = 0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            rank[k] += (hit[i] && (tn[i] < tn[k] || (tn[i] == tn[k] && i < k))) ? 1 : 0;
        ns += hit[k] ? 1 : 0;
    }
#pragma unroll
    for (int p = 0; p < KMAX; ++p) {
        sg.tn[p] = sg.tf[p] = 0.0;
        sg.tile[p] = 0;
        sg.n[p] = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (hit[k] && rank[k] == p) {
                sg.tn[p] = tn[k];
                sg.tf[p] = tf[k];
                sg.tile[p] = k;
            }
    }
    sg.ns = ns;
    if (ns == 0 || S_r <= 0) return;
    const int base = S_r >= ns ? 1 : 0;
    const int extra = S_r - base * ns;
    double total = 0.0;
#pragma unroll
    for (int p = 0; p < KMAX; ++p)
        if (p < ns) total += sg.tf[p] - sg.tn[p];
    double cum = 0.0;
    int prev = 0;
#pragma unroll
    for (int p = 0; p < KMAX; ++p) {
        if (p < ns) {
            cum += sg.tf[p] - sg.tn[p];
            const int b = (p == ns - 1) ? extra : (int)rint((double)extra * cum / total);
            sg.n[p] = base + b - prev;
            prev = b;
        }
    }
}

__device__ __forceinline__ void load_ray(const double *ro, const double *rd, int64_t r, double o[3],
                                         double d[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = ro[3 * r + a];
        d[a] = rd[3 * r + a];
    }
}

// ---- count ----------------------------------------------------------------
// Grouped = true also writes tcounts [K][R]: ray r's (kept) samples in tile k.
template <int KMAX, bool Grouped>
__global__ __launch_bounds__(256) void count_kernel(const double *__restrict__ ro,
                                                    const double *__restrict__ rd, int R, Boxes bx,
                                                    const int32_t *__restrict__ spr, int S,
                                                    const int32_t *__restrict__ max_count,
                                                    int32_t *__restrict__ counts,
                                                    float *__restrict__ view, int32_t *__restrict__ tcounts)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        double o[3], d[3];
        load_ray(ro, rd, r, o, d);
        Segs<KMAX> sg;
        int S_r = spr ? spr[r] : S;
        ray_segments<KMAX>(o, d, bx, S_r, sg);
        int c = 0;
#pragma unroll
        for (int p = 0; p < KMAX; ++p) c += sg.n[p];
        if (max_count) {
            int mc = max_count[r];
            mc = mc < 0 ? 0 : mc;
            c = mc < c ? mc : c;
        }
        counts[r] = c;
        if constexpr (Grouped) {
            // the kept prefix of c samples, segment by segment in entry order
            int per[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) per[k] = 0;
            int left = c;
#pragma unroll
            for (int p = 0; p < KMAX; ++p) {
                const int e = sg.n[p] < left ? sg.n[p] : left;
                left -= e;
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    if (p < sg.ns && sg.tile[p] == k) per[k] = e;
            }
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < bx.K) tcounts[(int64_t)k * R + r] = per[k];
        }
        if (view) {
            double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) view[3 * (int64_t)r + a] = (float)(d[a] / len);
        }
    }
}

// Where each tile's group starts: tile_start[k] = goffs[k][0] for k < K, and
// tile_start[K] = tile_start[K+1] = the total (no sample has a tile id >= K).
__global__ void tile_starts_kernel(const int32_t *__restrict__ goffs, int R, int K,
                                   const int64_t *__restrict__ total, int64_t *__restrict__ tile_start)
{
    const int k = threadIdx.x;
    if (k < K) tile_start[k] = R > 0 ? goffs[(int64_t)k * R] : 0;
    if (k == K || k == K + 1) tile_start[k] = R > 0 ? *total : 0;
}

// ---- fill: one wavefront per ray, one lane per sample -----------------------
//
// Grouped = false writes every sample at its packed (ray-major) index.
// Grouped = true writes t0/t1 there but pos, ray_id and tile_id grouped by
// tile -- tile by tile, ray by ray, in t within a ray (goffs [K][R]: where
// ray r's samples in tile k start) -- with smap[packed index] = grouped index.
template <int KMAX, bool Grouped>
__global__ __launch_bounds__(256) void fill_kernel(const double *__restrict__ ro,
                                                   const double *__restrict__ rd, int R, Boxes bx,
                                                   const int32_t *__restrict__ spr, int S,
                                                   const int32_t *__restrict__ info, int64_t cap,
                                                   float *__restrict__ t0, float *__restrict__ t1,
                                                   float *__restrict__ pos, int32_t *__restrict__ ray_id,
                                                   uint8_t *__restrict__ tile_id,
                                                   const int32_t *__restrict__ goffs, int32_t *__restrict__ smap)
{
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < R; r += waves) {
        const int64_t start = info[2 * (int64_t)r];
        const int count = info[2 * (int64_t)r + 1];
        if (count == 0) continue;
        // grouped form: where this ray's samples start in each tile's group,
        // tile k's in lane k (loaded first, so the load overlaps the segment
        // work; a sample reads its tile's with a lane shuffle)
        int32_t gl = 0;
        if constexpr (Grouped) {
            if (lane < bx.K) gl = goffs[(int64_t)lane * R + r];
        }
        double o[3], d[3];
        load_ray(ro, rd, r, o, d);
        Segs<KMAX> sg;
        int S_r = spr ? spr[r] : S;
        ray_segments<KMAX, true>(o, d, bx, S_r, sg);
        const int ns = sg.ns;
        // the tile-frame origin and direction of each segment's box: lane p
        // computes segment p's, and a sample reads them from that lane
        float olp[3], dlp[3];
        {
            int tp = sg.tile[0];
#pragma unroll
            for (int p = 1; p < KMAX; ++p)
                if (KMAX > 1 && lane == p) tp = sg.tile[p];
            // the whole box (the altitude band clips only the segment)
            double b[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) b[e] = bx.b[0][e];
#pragma unroll
            for (int t = 1; t < KMAX; ++t)
                if (tp == t) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) b[e] = bx.b[t][e];
                }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ext = b[3 + a] - b[a];
                olp[a] = (float)((o[a] - b[a]) / ext);
                dlp[a] = (float)(d[a] / ext);
            }
        }
        // every lane runs every trip, so that each one's segment values can
        // be read from any lane; a lane past the ray's count stores nothing
        for (int j0 = 0; j0 < count; j0 += 64) {
            const int j = j0 + lane;
            // segment of packed sample j: the first whose end lies past j, or the last
            int s = 0, before = 0;
#pragma unroll
            for (int p = 0; p + 1 < KMAX; ++p)
                if (s == p && p < ns - 1 && j >= before + sg.n[p]) {
                    before += sg.n[p];
                    s = p + 1;
                }
            double stn = sg.tn[0], stf = sg.tf[0];
            int n = sg.n[0], tile = sg.tile[0];
#pragma unroll
            for (int p = 1; p < KMAX; ++p)
                if (s == p) {
                    stn = sg.tn[p];
                    stf = sg.tf[p];
                    n = sg.n[p];
                    tile = sg.tile[p];
                }
            float ol[3], dl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ol[a] = KMAX > 1 ? __shfl(olp[a], s, 64) : olp[a];
                dl[a] = KMAX > 1 ? __shfl(dlp[a], s, 64) : dlp[a];
            }
            const int32_t gstart = Grouped ? __shfl(gl, tile, 64) : 0;
            if (j >= count) continue;
            const int k = j - before;
            float tn = (float)stn, tf = (float)stf;
            float step = (tf - tn) / (float)n;
            float ta = tn + (float)k * step;
            float tb = (k + 1 == n) ? tf : tn + (float)(k + 1) * step;
            float m = 0.5f * (ta + tb);
            const int64_t out = start + j;
            if (out >= cap) continue;
            t0[out] = ta;
            t1[out] = tb;
            int64_t g = out;
            if constexpr (Grouped) {
                g = (int64_t)gstart + k;
                // past the capacity (an overflow, flagged by the scan) the
                // map still points inside the arrays
                smap[out] = (int32_t)(g < cap ? g : cap - 1);
                if (g >= cap) continue;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float x = ol[a] + m * dl[a];
                x = x < 0.0f ? 0.0f : x;
                x = x > 1.0f ? 1.0f : x;
                pos[3 * g + a] = x;
            }
            ray_id[g] = r;
            if (tile_id) tile_id[g] = (uint8_t)tile;
        }
    }
}

// ---- early-stop index list --------------------------------------------------
__global__ __launch_bounds__(256) void alive_count_kernel(const int32_t *__restrict__ info,
                                                          const int32_t *__restrict__ n_alive, int R,
                                                          int32_t *__restrict__ counts)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        int c = info[2 * (int64_t)r + 1];
        int a = n_alive[r];
        a = a < 0 ? 0 : a;
        counts[r] = a < c ? a : c;
    }
}

__global__ __launch_bounds__(256) void alive_fill_kernel(const int32_t *__restrict__ info,
                                                         const int32_t *__restrict__ counts,
                                                         const int32_t *__restrict__ offs, int R,
                                                         int64_t cap, int32_t *__restrict__ idx_out)
{
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < R; r += waves) {
        const int32_t start = info[2 * (int64_t)r];
        const int c = counts[r];
        const int64_t o = offs[r];
        for (int j = lane; j < c; j += 64)
            if (o + j < cap) idx_out[o + j] = start + j;
    }
}

// Sliding-window acceptance (Sec. 4.4): the ray's chord through the band
// [z_lo, z_hi] (t >= 0) must be non-empty, bounded, and have both end points
// inside the closed rectangle win.  FP64, no contraction (file-wide), so the
// decision is the written arithmetic bit for bit.
struct Window {
    double x_lo, y_lo, x_hi, y_hi, z_lo, z_hi;
};

__device__ __forceinline__ int window_accepts(const double *o, const double *d, const Window &w)
{
    if (d[2] == 0.0) return 0;
    const double ta = (w.z_lo - o[2]) / d[2];
    const double tb = (w.z_hi - o[2]) / d[2];
    double t0 = ta < tb ? ta : tb;
    const double t1 = ta < tb ? tb : ta;
    if (t0 < 0.0) t0 = 0.0;
    if (!(t1 >= t0)) return 0;
    int ok = 1;
    const double ts[2] = {t0, t1};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const double x = o[0] + ts[e] * d[0];
        const double y = o[1] + ts[e] * d[1];
        if (!(x >= w.x_lo && x <= w.x_hi && y >= w.y_lo && y <= w.y_hi)) ok = 0;
    }
    return ok;
}

__global__ __launch_bounds__(256) void accept_count_kernel(const double *__restrict__ rays_o,
                                                           const double *__restrict__ rays_d, int R, Window w,
                                                           int32_t *__restrict__ counts,
                                                           uint8_t *__restrict__ accept)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        const double o[3] = {rays_o[3 * (int64_t)r], rays_o[3 * (int64_t)r + 1], rays_o[3 * (int64_t)r + 2]};
        const double d[3] = {rays_d[3 * (int64_t)r], rays_d[3 * (int64_t)r + 1], rays_d[3 * (int64_t)r + 2]};
        const int a = window_accepts(o, d, w);
        counts[r] = a;
        if (accept) accept[r] = (uint8_t)a;
    }
}

__global__ __launch_bounds__(256) void accept_fill_kernel(const int32_t *__restrict__ counts,
                                                          const int32_t *__restrict__ offs, int R,
                                                          int32_t *__restrict__ idx_out)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x)
        if (counts[r]) idx_out[offs[r]] = r;
}

__global__ void set_i64_kernel(int64_t *p, int64_t v) { *p = v; }

// workspace: counts[R] | offs[R] | bsum[nb]
// ---- density-driven refinement after culling (Sec. 4.1) ---------------------
// A ray whose culled set holds c > 0 intervals spends its whole budget B (its
// sample count before culling) on them: interval i gets e(i+1) - e(i) equal
// sub-intervals, e(i) = floor((2 B i + c) / (2 c)); a ray that keeps nothing
// gets no samples.  The sub-interval bounds and the midpoint's tile-frame
// position use the fill kernel's rounding points.
__global__ __launch_bounds__(256) void refine_count_kernel(const int32_t *__restrict__ info_all,
                                                           const int32_t *__restrict__ info_kept, int R,
                                                           int32_t *__restrict__ counts)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x)
        counts[r] = info_kept[2 * (int64_t)r + 1] > 0 ? info_all[2 * (int64_t)r + 1] : 0;
}

__device__ __forceinline__ int64_t split_edge(int64_t B, int64_t c, int64_t i) { return (2 * B * i + c) / (2 * c); }

// One wavefront per ray, one lane per refined sample.
template <int KMAX>
__global__ __launch_bounds__(256) void refine_fill_kernel(const double *__restrict__ ro, const double *__restrict__ rd,
                                                          int R, Boxes bx, const int32_t *__restrict__ info_kept,
                                                          const float *__restrict__ t0k, const float *__restrict__ t1k,
                                                          const uint8_t *__restrict__ tilek,
                                                          const int32_t *__restrict__ info, int64_t cap,
                                                          float *__restrict__ t0, float *__restrict__ t1,
                                                          float *__restrict__ pos, int32_t *__restrict__ ray_id,
                                                          uint8_t *__restrict__ tile_id)
{
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < R; r += waves) {
        const int64_t sk = info_kept[2 * (int64_t)r];
        const int64_t c = info_kept[2 * (int64_t)r + 1];
        const int64_t start = info[2 * (int64_t)r];
        const int64_t B = info[2 * (int64_t)r + 1];
        if (B == 0 || c == 0) continue;
        double o[3], d[3];
        load_ray(ro, rd, r, o, d);
        for (int64_t j = lane; j < B; j += 64) {
            // the kept interval holding refined sample j: the last i with e(i) <= j
            int64_t i = j * c / B;
            while (i + 1 < c && split_edge(B, c, i + 1) <= j) ++i;
            while (i > 0 && split_edge(B, c, i) > j) --i;
            const int64_t e0 = split_edge(B, c, i);
            const int64_t q = split_edge(B, c, i + 1) - e0, k = j - e0;
            const float ta = t0k[sk + i], tb = t1k[sk + i];
            const int tile = tilek ? tilek[sk + i] : 0;
            double b[6] = {bx.b[0][0], bx.b[0][1], bx.b[0][2], bx.b[0][3], bx.b[0][4], bx.b[0][5]};
#pragma unroll
            for (int t = 1; t < KMAX; ++t)
                if (tile == t) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) b[e] = bx.b[t][e];
                }
            const float h = (tb - ta) / (float)q;
            const float ta2 = ta + (float)k * h;
            const float tb2 = (k + 1 == q) ? tb : ta + (float)(k + 1) * h;
            const float m = 0.5f * (ta2 + tb2);
            const int64_t out = start + j;
            if (out >= cap) continue;
            t0[out] = ta2;
            t1[out] = tb2;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ext = b[3 + a] - b[a];
                const float ol = (float)((o[a] - b[a]) / ext);
                const float dl = (float)(d[a] / ext);
                float x = ol + m * dl;
                x = x < 0.0f ? 0.0f : x;
                x = x > 1.0f ? 1.0f : x;
                pos[3 * out + a] = x;
            }
            ray_id[out] = r;
            if (tile_id) tile_id[out] = (uint8_t)tile;
        }
    }
}

struct ScanWs {
    int32_t *counts, *offs;
    int64_t *bsum;
    int nb;
};

size_t scan_ws_bytes(int32_t R)
{
    size_t r = (size_t)(R > 0 ? R : 1);
    size_t nb = (size_t)scan::scan_blocks((int64_t)r);
    return 2 * ((r * 4 + 255) / 256 * 256) + nb * 8 + 256;
}

ScanWs carve(void *ws, int32_t R)
{
    size_t r = (size_t)(R > 0 ? R : 1);
    size_t a = (r * 4 + 255) / 256 * 256;
    char *p = static_cast<char *>(ws);
    ScanWs s;
    s.counts = reinterpret_cast<int32_t *>(p);
    s.offs = reinterpret_cast<int32_t *>(p + a);
    s.bsum = reinterpret_cast<int64_t *>(p + 2 * a);
    s.nb = scan::scan_blocks((int64_t)r);
    return s;
}

void launch_scan(const ScanWs &w, int R, int32_t *start, int stride, int32_t *count_dst, int64_t cap,
                 int64_t *n_out, hipStream_t st)
{
    scan::launch_scan(w.counts, R, w.bsum, start, stride, count_dst, cap, n_out, device_error_word(), st);
}

}  // namespace
}  // namespace snake

using namespace snake;

extern "C" {

size_t snake_sample_workspace_bytes(int32_t R) { return scan_ws_bytes(R); }

// The sampler on a given count/scan workspace; fn names the entry point in
// error messages.
static size_t grouped_ws_bytes(int32_t R, int32_t K)
{
    return scan_ws_bytes(R) + scan_ws_bytes(R * K) + 256;
}

// smap != NULL: the grouped form (pos, ray_id, tile_id grouped by tile,
// smap and tile_start written; the workspace as grouped_ws_bytes).
static int sample_impl(const char *fn, const double *rays_o, const double *rays_d, int32_t R, const double *boxes,
                       int32_t K, const double *zband, const int32_t *samples_per_ray, int32_t S,
                       const int32_t *max_count, int32_t *packed_info, float *t0, float *t1, float *pos,
                       int32_t *ray_id, uint8_t *tile_id, float *view, int64_t cap, int64_t *n_out,
                       void *workspace, size_t workspace_bytes, snake_stream_t stream, int32_t *smap = nullptr,
                       int64_t *tile_start = nullptr)
{
    const bool grouped = smap != nullptr;
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "%s: R = %d < 0", fn, R);
    SNAKE_REQUIRE(K >= 1 && K <= kMaxTiles, SNAKE_ERR_INVALID_ARG, "%s: K = %d not in [1, %d]", fn, K, kMaxTiles);
    SNAKE_REQUIRE(K == 1 || tile_id != nullptr, SNAKE_ERR_NULL, "%s: tile_id is NULL with K = %d > 1", fn, K);
    SNAKE_REQUIRE(samples_per_ray != nullptr || S >= 0, SNAKE_ERR_INVALID_ARG, "%s: S = %d < 0", fn, S);
    SNAKE_REQUIRE(cap >= 0 && cap <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "%s: cap = %lld not in [0, 2^31)", fn,
                  (long long)cap);
    SNAKE_REQUIRE(boxes != nullptr && n_out != nullptr, SNAKE_ERR_NULL, "%s: boxes or n_out is NULL", fn);
    SNAKE_REQUIRE(R == 0 || (rays_o && rays_d && packed_info), SNAKE_ERR_NULL,
                  "%s: rays_o, rays_d or packed_info is NULL", fn);
    SNAKE_REQUIRE(cap == 0 || (t0 && t1 && pos && ray_id), SNAKE_ERR_NULL, "%s: t0, t1, pos or ray_id is NULL", fn);
    if (grouped) {
        SNAKE_REQUIRE((int64_t)R * K <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "%s: R * K = %lld not below 2^31", fn,
                      (long long)R * K);
        SNAKE_REQUIRE(tile_start != nullptr && tile_id != nullptr, SNAKE_ERR_NULL, "%s: tile_start or tile_id is NULL",
                      fn);
    }
    const size_t need = grouped ? grouped_ws_bytes(R, K) : scan_ws_bytes(R);
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= need, SNAKE_ERR_WORKSPACE, "%s: workspace needs %zu bytes",
                  fn, need);
    SNAKE_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % 256 == 0, SNAKE_ERR_ALIGN,
                  "%s: workspace is not 256-byte aligned", fn);
    Boxes bx{};
    bx.K = K;
    for (int k = 0; k < K; ++k) {
        for (int a = 0; a < 6; ++a) bx.b[k][a] = boxes[6 * k + a];
        for (int a = 0; a < 3; ++a)
            SNAKE_REQUIRE(bx.b[k][3 + a] > bx.b[k][a], SNAKE_ERR_INVALID_ARG, "%s: box %d is empty on axis %d", fn,
                          k, a);
    }
    if (zband) {
        SNAKE_REQUIRE(zband[1] > zband[0], SNAKE_ERR_INVALID_ARG, "%s: empty altitude band", fn);
        bx.use_band = 1;
        bx.z_lo = zband[0];
        bx.z_hi = zband[1];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (R == 0) {
        set_i64_kernel<<<1, 1, 0, st>>>(n_out, 0);
        if (grouped) tile_starts_kernel<<<1, 64, 0, st>>>(nullptr, 0, K, nullptr, tile_start);
        return launch_status(fn);
    }
    ScanWs w = carve(workspace, R);
    // the grouped form's per-tile counts and their scan, after the ray scan's
    ScanWs tw{};
    int64_t *gtotal = nullptr;
    if (grouped) {
        char *p = static_cast<char *>(workspace) + scan_ws_bytes(R);
        tw = carve(p, R * K);
        gtotal = reinterpret_cast<int64_t *>(p + scan_ws_bytes(R * K));
    }
    const unsigned gc = grid_for(R, 256, 8), gf = grid_for((int64_t)R * 64, 256, tune(SNAKE_TUNE_SAMPLER_BLOCKS_PER_CU));
#define SNAKE_SAMPLER_LAUNCH(KM)                                                                              \
    if (grouped) {                                                                                            \
        count_kernel<KM, true><<<gc, 256, 0, st>>>(rays_o, rays_d, R, bx, samples_per_ray, S, max_count,      \
                                                   w.counts, view, tw.counts);                               \
        launch_scan(w, R, packed_info, 2, packed_info + 1, cap, n_out, st);                                   \
        launch_scan(tw, R * K, tw.offs, 1, nullptr, cap, gtotal, st);                                         \
        tile_starts_kernel<<<1, 64, 0, st>>>(tw.offs, R, K, gtotal, tile_start);                              \
        fill_kernel<KM, true><<<gf, 256, 0, st>>>(rays_o, rays_d, R, bx, samples_per_ray, S, packed_info,     \
                                                  cap, t0, t1, pos, ray_id, tile_id, tw.offs, smap);          \
    } else {                                                                                                  \
        count_kernel<KM, false><<<gc, 256, 0, st>>>(rays_o, rays_d, R, bx, samples_per_ray, S, max_count,     \
                                                    w.counts, view, nullptr);                                \
        launch_scan(w, R, packed_info, 2, packed_info + 1, cap, n_out, st);                                   \
        fill_kernel<KM, false><<<gf, 256, 0, st>>>(rays_o, rays_d, R, bx, samples_per_ray, S, packed_info,    \
                                                   cap, t0, t1, pos, ray_id, tile_id, nullptr, nullptr);      \
    }
    if (K == 1) {
        SNAKE_SAMPLER_LAUNCH(1);
    } else if (K <= 4) {
        SNAKE_SAMPLER_LAUNCH(4);
    } else {
        SNAKE_SAMPLER_LAUNCH(kMaxTiles);
    }
#undef SNAKE_SAMPLER_LAUNCH
    return launch_status(fn);
}

// The no-allocation variant's scratch: the count/scan workspace for up to
// kStaticRays rays in one file-scope device array (each device holds its own
// copy until the process ends).  Host code never uses the array's name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
constexpr int32_t kStaticRays = 1 << 20;
constexpr size_t kStaticScratchBytes =
    2 * (((size_t)kStaticRays * 4 + 255) / 256 * 256) + ((size_t)kStaticRays / scan::kScanTile + 1) * 8 + 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static constexpr int kScratchDevices = 64;
static void *g_scratch[kScratchDevices];
static std::mutex g_scratch_mu;

// Device address of this device's scratch (the current device), resolved on
// the first call on that device; nullptr (with the error message set) on failure.
static void *scratch_address(const char *fn)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
        set_error("%s: no usable current device", fn);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("%s: hipGetSymbolAddress of the static scratch failed: %s", fn, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

int snake_sample_segmented(const double *rays_o, const double *rays_d, int32_t R, const double *boxes,
                           int32_t K, const double *zband, const int32_t *samples_per_ray, int32_t S,
                           const int32_t *max_count, int32_t *packed_info, float *t0, float *t1,
                           float *pos, int32_t *ray_id, uint8_t *tile_id, float *view, int64_t cap,
                           int64_t *n_out, void *workspace, size_t workspace_bytes,
                           snake_stream_t stream)
{
    return sample_impl(__func__, rays_o, rays_d, R, boxes, K, zband, samples_per_ray, S, max_count, packed_info, t0,
                       t1, pos, ray_id, tile_id, view, cap, n_out, workspace, workspace_bytes, stream);
}

size_t snake_sample_grouped_workspace_bytes(int32_t R, int32_t K)
{
    if (R < 0 || K < 1 || K > kMaxTiles || (int64_t)R * K > INT32_MAX) return 0;
    return grouped_ws_bytes(R, K);
}

int snake_sample_grouped(const double *rays_o, const double *rays_d, int32_t R, const double *boxes, int32_t K,
                         const double *zband, const int32_t *samples_per_ray, int32_t S, const int32_t *max_count,
                         int32_t *packed_info, float *t0, float *t1, float *view, float *pos, int32_t *ray_id,
                         uint8_t *tile_id, int32_t *sample_map, int64_t *tile_start, int64_t cap, int64_t *n_out,
                         void *workspace, size_t workspace_bytes, snake_stream_t stream)
{
    SNAKE_REQUIRE(cap == 0 || sample_map != nullptr, SNAKE_ERR_NULL, "snake_sample_grouped: sample_map is NULL");
    int32_t dummy = 0;
    return sample_impl(__func__, rays_o, rays_d, R, boxes, K, zband, samples_per_ray, S, max_count, packed_info, t0,
                       t1, pos, ray_id, tile_id, view, cap, n_out, workspace, workspace_bytes, stream,
                       sample_map ? sample_map : &dummy, tile_start);
}

int32_t snake_sample_segmented_static_max_rays(void) { return kStaticRays; }

int snake_sample_segmented_static(const double *rays_o, const double *rays_d, int32_t R, const double *boxes,
                                  int32_t K, const double *zband, const int32_t *samples_per_ray, int32_t S,
                                  const int32_t *max_count, int32_t *packed_info, float *t0, float *t1,
                                  float *pos, int32_t *ray_id, uint8_t *tile_id, float *view, int64_t cap,
                                  int64_t *n_out, snake_stream_t stream)
{
    SNAKE_REQUIRE(R <= kStaticRays, SNAKE_ERR_INVALID_ARG,
                  "snake_sample_segmented_static: R = %d exceeds the static scratch limit of %d rays", R,
                  kStaticRays);
    void *ws = scratch_address(__func__);
    if (!ws) return SNAKE_ERR_HIP;
    return sample_impl(__func__, rays_o, rays_d, R, boxes, K, zband, samples_per_ray, S, max_count, packed_info, t0,
                       t1, pos, ray_id, tile_id, view, cap, n_out, ws, kStaticScratchBytes, stream);
}

int snake_sample_refine(const double *rays_o, const double *rays_d, int32_t R, const double *boxes, int32_t K,
                        const int32_t *packed_info_all, const int32_t *packed_info_kept, const float *t0_kept,
                        const float *t1_kept, const uint8_t *tile_id_kept, int32_t *packed_info, float *t0,
                        float *t1, float *pos, int32_t *ray_id, uint8_t *tile_id, int64_t cap, int64_t *n_out,
                        void *workspace, size_t workspace_bytes, snake_stream_t stream)
{
    const char *fn = __func__;
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "%s: R = %d < 0", fn, R);
    SNAKE_REQUIRE(K >= 1 && K <= kMaxTiles, SNAKE_ERR_INVALID_ARG, "%s: K = %d not in [1, %d]", fn, K, kMaxTiles);
    SNAKE_REQUIRE(K == 1 || tile_id_kept != nullptr, SNAKE_ERR_NULL, "%s: tile_id_kept is NULL with K = %d > 1", fn,
                  K);
    SNAKE_REQUIRE(cap >= 0 && cap <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "%s: cap = %lld not in [0, 2^31)", fn,
                  (long long)cap);
    SNAKE_REQUIRE(boxes != nullptr && n_out != nullptr, SNAKE_ERR_NULL, "%s: boxes or n_out is NULL", fn);
    SNAKE_REQUIRE(R == 0 || (rays_o && rays_d && packed_info_all && packed_info_kept && t0_kept && t1_kept &&
                             packed_info),
                  SNAKE_ERR_NULL, "%s: an input array or packed_info is NULL", fn);
    SNAKE_REQUIRE(cap == 0 || (t0 && t1 && pos && ray_id), SNAKE_ERR_NULL, "%s: t0, t1, pos or ray_id is NULL", fn);
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= scan_ws_bytes(R), SNAKE_ERR_WORKSPACE,
                  "%s: workspace needs %zu bytes", fn, scan_ws_bytes(R));
    SNAKE_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % 256 == 0, SNAKE_ERR_ALIGN,
                  "%s: workspace is not 256-byte aligned", fn);
    Boxes bx{};
    bx.K = K;
    for (int k = 0; k < K; ++k) {
        for (int a = 0; a < 6; ++a) bx.b[k][a] = boxes[6 * k + a];
        for (int a = 0; a < 3; ++a)
            SNAKE_REQUIRE(bx.b[k][3 + a] > bx.b[k][a], SNAKE_ERR_INVALID_ARG, "%s: box %d is empty on axis %d", fn,
                          k, a);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (R == 0) {
        set_i64_kernel<<<1, 1, 0, st>>>(n_out, 0);
        return launch_status(fn);
    }
    ScanWs w = carve(workspace, R);
    const unsigned gc = grid_for(R, 256, 8), gf = grid_for((int64_t)R * 64, 256, tune(SNAKE_TUNE_SAMPLER_BLOCKS_PER_CU));
    refine_count_kernel<<<gc, 256, 0, st>>>(packed_info_all, packed_info_kept, R, w.counts);
    launch_scan(w, R, packed_info, 2, packed_info + 1, cap, n_out, st);
#define SNAKE_REFINE_LAUNCH(KM)                                                                                  \
    refine_fill_kernel<KM><<<gf, 256, 0, st>>>(rays_o, rays_d, R, bx, packed_info_kept, t0_kept, t1_kept,      \
                                               tile_id_kept, packed_info, cap, t0, t1, pos, ray_id, tile_id)
    if (K == 1) {
        SNAKE_REFINE_LAUNCH(1);
    } else if (K <= 4) {
        SNAKE_REFINE_LAUNCH(4);
    } else {
        SNAKE_REFINE_LAUNCH(kMaxTiles);
    }
#undef SNAKE_REFINE_LAUNCH
    return launch_status(fn);
}

int snake_pack_alive(const int32_t *packed_info, const int32_t *n_alive, int32_t R, int32_t *idx_out,
                     int64_t cap, int64_t *n_out, void *workspace, size_t workspace_bytes,
                     snake_stream_t stream)
{
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "snake_pack_alive: R = %d < 0", R);
    SNAKE_REQUIRE(cap >= 0 && cap <= INT32_MAX, SNAKE_ERR_INVALID_ARG, "snake_pack_alive: bad cap");
    SNAKE_NOT_NULL(n_out);
    if (R > 0) {
        SNAKE_NOT_NULL(packed_info);
        SNAKE_NOT_NULL(n_alive);
    }
    if (cap > 0) SNAKE_NOT_NULL(idx_out);
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= scan_ws_bytes(R), SNAKE_ERR_WORKSPACE,
                  "snake_pack_alive: workspace needs %zu bytes", scan_ws_bytes(R));
    SNAKE_ALIGNED(workspace, 256);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (R == 0) {
        set_i64_kernel<<<1, 1, 0, st>>>(n_out, 0);
        return launch_status(__func__);
    }
    ScanWs w = carve(workspace, R);
    alive_count_kernel<<<grid_for(R, 256, 8), 256, 0, st>>>(packed_info, n_alive, R, w.counts);
    launch_scan(w, R, w.offs, 1, nullptr, cap, n_out, st);
    alive_fill_kernel<<<grid_for((int64_t)R * 64, 256, 16), 256, 0, st>>>(packed_info, w.counts, w.offs,
                                                                         R, cap, idx_out);
    return launch_status(__func__);
}

int snake_window_accept(const double *rays_o, const double *rays_d, int32_t R, const double *window,
                        const double *zband, uint8_t *accept, int32_t *idx_out, int64_t *n_out,
                        void *workspace, size_t workspace_bytes, snake_stream_t stream)
{
    SNAKE_REQUIRE(R >= 0, SNAKE_ERR_INVALID_ARG, "snake_window_accept: R = %d < 0", R);
    SNAKE_NOT_NULL(window);
    SNAKE_NOT_NULL(zband);
    SNAKE_NOT_NULL(n_out);
    Window w{window[0], window[1], window[2], window[3], zband[0], zband[1]};
    SNAKE_REQUIRE(w.x_lo <= w.x_hi && w.y_lo <= w.y_hi && w.z_lo <= w.z_hi, SNAKE_ERR_INVALID_ARG,
                  "snake_window_accept: empty window or band");
    if (R > 0) {
        SNAKE_NOT_NULL(rays_o);
        SNAKE_NOT_NULL(rays_d);
        SNAKE_NOT_NULL(idx_out);
    }
    SNAKE_REQUIRE(workspace != nullptr && workspace_bytes >= scan_ws_bytes(R), SNAKE_ERR_WORKSPACE,
                  "snake_window_accept: workspace needs %zu bytes", scan_ws_bytes(R));
    SNAKE_ALIGNED(workspace, 256);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (R == 0) {
        set_i64_kernel<<<1, 1, 0, st>>>(n_out, 0);
        return launch_status(__func__);
    }
    ScanWs ws = carve(workspace, R);
    accept_count_kernel<<<grid_for(R, 256, 8), 256, 0, st>>>(rays_o, rays_d, R, w, ws.counts, accept);
    launch_scan(ws, R, ws.offs, 1, nullptr, R, n_out, st);
    accept_fill_kernel<<<grid_for(R, 256, 8), 256, 0, st>>>(ws.counts, ws.offs, R, idx_out);
    return launch_status(__func__);
}

}  // extern "C"
