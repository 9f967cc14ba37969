/*
 * CPU FP64 oracle for one training step of a tile NeRF (Snake-NeRF,
 * "Tile and Slide", arXiv 2507.01631).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled with gcc and is called
 * by the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  It shares no code, header or constant with the HIP library,
 * and the library never calls it.
 *
 * Plain, slow and obviously correct: FP64 everywhere except at the FP32
 * rounding points that the library boundary itself defines (sample bounds,
 * sample positions, hash-grid cell coordinates).  Those rounding points are
 * what make sample bounds and hash indices comparable bit for bit.
 *
 * What each function follows:
 *   - orc_sample_segmented: the segmented sampler of Sec. 4.5 (near/far per
 *     NeRF tile, samples drawn separately on each segment so that adjacent
 *     segments meet exactly on the shared box face), with the UTM-to-local
 *     mapping of Sec. 4.1-4.2 (tile box -> [0,1]^3) and the per-ray segment
 *     distribution of Sec. 4.6.
 *   - orc_window_accept: which rays a loaded 2x2 window of NeRF tiles may
 *     train on (Sec. 4.4, sliding window).
 *   - orc_hashgrid_*: the multiresolution hash encoding the paper adopts in
 *     Sec. 4.1 (the NGP representation it cites): per level a grid of
 *     resolution N_l, the 8 cell corners, dense indexing when the grid fits
 *     the table, else the prime-XOR spatial hash, trilinear blend.
 *   - orc_mlp_*: the local density network (sigma + density embedding) and
 *     the colour network fed by the embedding, Sec. 4.1.
 *   - orc_composite_*: the unmodified NeRF volume-rendering quadrature the
 *     paper keeps (Sec. 2.2 and Sec. 4.5) and the colour-consistency (MSE)
 *     loss of Sec. 4.4.
 *   - orc_adam_step: the optimiser of the I-NGP training strategy the paper
 *     states it shares (Sec. 4.6).
 * Readings where the paper is silent are listed in the design notes.
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 * (no FMA contraction, so every rounding point below is the written one).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_TILES 64
#define ORC_MAX_LEVELS 32

/* ------------------------------------------------------------------ */
/* Level resolutions                                                   */
/* ------------------------------------------------------------------ */

/* N_l = floor(N_min * b^l + 1e-6), b = exp(ln(N_max/N_min)/(L-1)): the
 * geometric level rule of the cited hash encoding.  L = 1 gives N_min. */
void orc_level_resolutions(int L, int n_min, int n_max, int32_t *res)
{
    double b = (L > 1) ? exp(log((double)n_max / (double)n_min) / (double)(L - 1)) : 1.0;
    for (int l = 0; l < L; ++l)
        res[l] = (int32_t)floor((double)n_min * pow(b, (double)l) + 1e-6);
}

/* ------------------------------------------------------------------ */
/* Segmented sampler                                                   */
/* ------------------------------------------------------------------ */

/* Slab test of a ray against an axis-aligned box, in FP64.
 * Returns 1 and the chord [t_near, t_far] (t_near clamped at 0) when
 * t_far > t_near, 0 otherwise: a ray that only touches an edge or a corner
 * is a miss.  A ray parallel to an axis (d_a == 0) is inside that slab when
 * lo_a <= o_a < hi_a: half-open, so that a ray lying in the face shared by
 * two neighbouring boxes belongs to exactly one of them. */
static int slab(const double o[3], const double d[3], const double lo[3],
                const double hi[3], double *tn, double *tf)
{
    double t_near = -INFINITY, t_far = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] >= hi[a]) return 0;
            continue;
        }
        double t_lo = (lo[a] - o[a]) / d[a];
        double t_hi = (hi[a] - o[a]) / d[a];
        double a_min = t_lo < t_hi ? t_lo : t_hi;
        double a_max = t_lo < t_hi ? t_hi : t_lo;
        if (a_min > t_near) t_near = a_min;
        if (a_max < t_far) t_far = a_max;
    }
    if (t_near < 0.0) t_near = 0.0;
    if (!(t_far > t_near)) return 0;
    *tn = t_near;
    *tf = t_far;
    return 1;
}

typedef struct { double tn, tf; int tile; int n; } orc_seg;

/* Segments of one ray over the K NeRF tiles, sorted by entry distance, and
 * the share of the ray's sample budget S_r each one receives.  When
 * S_r >= n_seg every segment first gets one sample (so the segments' near and
 * far bounds all appear as sample bounds and the samples cover the whole
 * chord); the remaining E = S_r - n_seg samples are split in proportion to
 * segment length by cumulative rounding, b_s = rint(E * cum_s / total),
 * n_s = 1 + b_s - b_{s-1}.  With S_r < n_seg the whole budget is split that
 * way with no minimum.  Either way sum n_s = S_r. */
static int ray_segments(const double o[3], const double d[3], int K,
                        const double *boxes, const double *zband, int S_r,
                        orc_seg *segs)
{
    int n = 0;
    for (int k = 0; k < K; ++k) {
        double lo[3] = {boxes[6 * k + 0], boxes[6 * k + 1], boxes[6 * k + 2]};
        double hi[3] = {boxes[6 * k + 3], boxes[6 * k + 4], boxes[6 * k + 5]};
        if (zband) {
            if (zband[0] > lo[2]) lo[2] = zband[0];
            if (zband[1] < hi[2]) hi[2] = zband[1];
        }
        double tn, tf;
        if (slab(o, d, lo, hi, &tn, &tf)) {
            segs[n].tn = tn;
            segs[n].tf = tf;
            segs[n].tile = k;
            segs[n].n = 0;
            ++n;
        }
    }
    /* insertion sort by entry distance (ties broken by tile index) */
    for (int i = 1; i < n; ++i) {
        orc_seg s = segs[i];
        int j = i - 1;
        while (j >= 0 && (segs[j].tn > s.tn || (segs[j].tn == s.tn && segs[j].tile > s.tile))) {
            segs[j + 1] = segs[j];
            --j;
        }
        segs[j + 1] = s;
    }
    if (n == 0 || S_r <= 0) return n;
    int base = S_r >= n ? 1 : 0;
    int E = S_r - base * n;
    double total = 0.0;
    for (int i = 0; i < n; ++i) total += segs[i].tf - segs[i].tn;
    double cum = 0.0;
    int prev = 0;
    for (int i = 0; i < n; ++i) {
        cum += segs[i].tf - segs[i].tn;
        int b = (i == n - 1) ? E : (int)rint((double)E * cum / total);
        segs[i].n = base + b - prev;
        prev = b;
    }
    return n;
}

/*
 * For every ray r: segments through the K boxes (optionally clipped to the
 * altitude band zband = [z_lo, z_hi]), S_r = samples_per_ray ? spr[r] : S
 * samples split over them, optionally truncated to max_count[r].  Samples of
 * a ray are contiguous and ordered by t; packed_info[r] = (start, count).
 *
 * Sample j of a segment with n samples is the interval [t_j, t_{j+1}] with
 *   tn = fl32(t_near), tf = fl32(t_far), step = fl32(fl32(tf - tn) / n),
 *   t_j = fl32(tn + fl32(j * step)) for j < n, and t_n = tf,
 * evaluated at its midpoint m = fl32(0.5 * fl32(t_j + t_{j+1})) whose
 * position in the tile's [0,1]^3 frame is
 *   pos_a = clamp(fl32(o_a' + fl32(m * d_a')), 0, 1),
 *   o_a' = fl32((o_a - lo_a) / (hi_a - lo_a)),  d_a' = fl32(d_a / (hi_a - lo_a)).
 * view[r] = fl32(d / |d|).
 * Returns 0, or -1 when the packed total exceeds cap (outputs then hold
 * only packed_info and *n_out, the required total).
 */
int orc_sample_segmented(int R, const double *rays_o, const double *rays_d,
                         int K, const double *boxes, const double *zband,
                         const int32_t *samples_per_ray, int S,
                         const int32_t *max_count,
                         int32_t *packed_info, float *t0, float *t1, float *pos,
                         int32_t *ray_id, uint8_t *tile_id, float *view,
                         int64_t cap, int64_t *n_out)
{
    if (K < 1 || K > ORC_MAX_TILES) return -2;
    int64_t total = 0;
    for (int r = 0; r < R; ++r) {
        orc_seg segs[ORC_MAX_TILES];
        int S_r = samples_per_ray ? samples_per_ray[r] : S;
        int ns = ray_segments(rays_o + 3 * r, rays_d + 3 * r, K, boxes, zband, S_r, segs);
        int count = 0;
        for (int s = 0; s < ns; ++s) count += segs[s].n;
        if (max_count && max_count[r] < count) count = max_count[r] < 0 ? 0 : max_count[r];
        packed_info[2 * r + 0] = (int32_t)total;
        packed_info[2 * r + 1] = count;
        total += count;
    }
    *n_out = total;
    if (total > cap) return -1;

#pragma omp parallel for schedule(dynamic, 64)
    for (int r = 0; r < R; ++r) {
        const double *o = rays_o + 3 * r, *d = rays_d + 3 * r;
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; ++a) view[3 * r + a] = (float)(d[a] / len);

        orc_seg segs[ORC_MAX_TILES];
        int S_r = samples_per_ray ? samples_per_ray[r] : S;
        int ns = ray_segments(o, d, K, boxes, zband, S_r, segs);
        int64_t out = packed_info[2 * r + 0];
        int left = packed_info[2 * r + 1];
        for (int s = 0; s < ns && left > 0; ++s) {
            int n = segs[s].n;
            if (n == 0) continue;
            const double *b = boxes + 6 * segs[s].tile;
            float ol[3], dl[3];
            for (int a = 0; a < 3; ++a) {
                double ext = b[3 + a] - b[a];
                ol[a] = (float)((o[a] - b[a]) / ext);
                dl[a] = (float)(d[a] / ext);
            }
            float tn = (float)segs[s].tn, tf = (float)segs[s].tf;
            float step = (tf - tn) / (float)n;
            for (int j = 0; j < n && left > 0; ++j, --left, ++out) {
                float ta = tn + (float)j * step;
                float tb = (j + 1 == n) ? tf : tn + (float)(j + 1) * step;
                float m = 0.5f * (ta + tb);
                t0[out] = ta;
                t1[out] = tb;
                for (int a = 0; a < 3; ++a) {
                    float x = ol[a] + m * dl[a];
                    if (x < 0.0f) x = 0.0f;
                    if (x > 1.0f) x = 1.0f;
                    pos[3 * out + a] = x;
                }
                ray_id[out] = r;
                tile_id[out] = (uint8_t)segs[s].tile;
            }
        }
    }
    return 0;
}

/*
 * Ray acceptance of the 2x2 sliding window (Sec. 4.4): a ray is used while
 * the window is loaded only if every NeRF tile it crosses is one of the
 * window's tiles.  The tiles of a window share the altitude band
 * [z_lo, z_hi] and together cover the rectangle win = [x_lo, x_hi] x
 * [y_lo, y_hi], so the test is: the part of the ray (t >= 0) inside the band
 * is non-empty and bounded, and both of its end points have x, y inside the
 * closed rectangle (the chord is a segment and the rectangle convex, so the
 * whole chord is then inside).  A ray parallel to the band planes is
 * rejected (its chord is unbounded).  accept[r] = 1 or 0; returns the count.
 */
int64_t orc_window_accept(int R, const double *rays_o, const double *rays_d,
                          const double win[4], double z_lo, double z_hi, int32_t *accept)
{
    int64_t n = 0;
    for (int r = 0; r < R; ++r) {
        const double *o = rays_o + 3 * r, *d = rays_d + 3 * r;
        int ok = 0;
        if (d[2] != 0.0) {
            double ta = (z_lo - o[2]) / d[2];
            double tb = (z_hi - o[2]) / d[2];
            double t0 = ta < tb ? ta : tb;
            double t1 = ta < tb ? tb : ta;
            if (t0 < 0.0) t0 = 0.0;
            if (t1 >= t0) {
                ok = 1;
                double ts[2] = {t0, t1};
                for (int e = 0; e < 2; ++e) {
                    double x = o[0] + ts[e] * d[0];
                    double y = o[1] + ts[e] * d[1];
                    if (!(x >= win[0] && x <= win[2] && y >= win[1] && y <= win[3])) ok = 0;
                }
            }
        }
        accept[r] = ok;
        n += ok;
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Hash grid                                                           */
/* ------------------------------------------------------------------ */

/* Table slot of integer grid corner (i,j,k) at a level of resolution N:
 * dense row-major (x fastest) when (N+1)^3 <= T, otherwise the spatial hash
 * (i*1 XOR j*2654435761 XOR k*805459861) mod 2^32, reduced mod T. */
uint32_t orc_hash_index(uint32_t i, uint32_t j, uint32_t k, int N, int log2T, int always_hash)
{
    uint64_t T = (uint64_t)1 << log2T;
    uint64_t side = (uint64_t)N + 1;
    if (!always_hash && side * side * side <= T)
        return (uint32_t)(i + j * side + k * side * side);
    uint32_t h = (i * 1u) ^ (j * 2654435761u) ^ (k * 805459861u);
    return h & (uint32_t)(T - 1);
}

/* Cell of x in a level of resolution N: p = fl32(x * N), c = min(floor p, N-1),
 * w = p - c (exact in FP32).  x = 1 therefore lands on weight 1 of the last cell. */
static void cell(float x, int N, uint32_t *c, double *w)
{
    float p = x * (float)N;
    float f = floorf(p);
    if (f > (float)(N - 1)) f = (float)(N - 1);
    if (f < 0.0f) f = 0.0f;
    *c = (uint32_t)f;
    *w = (double)(p - f);
}

/* The 8 corner slots and trilinear weights of point x at level l.  Corner c
 * uses bit 0 for x, bit 1 for y, bit 2 for z; weight = prod_a (bit ? w_a : 1-w_a). */
void orc_hash_corners(const float x[3], int N, int log2T, int always_hash,
                      uint32_t idx[8], double wgt[8])
{
    uint32_t c[3];
    double w[3];
    for (int a = 0; a < 3; ++a) cell(x[a], N, &c[a], &w[a]);
    for (int q = 0; q < 8; ++q) {
        int bx = q & 1, by = (q >> 1) & 1, bz = (q >> 2) & 1;
        idx[q] = orc_hash_index(c[0] + bx, c[1] + by, c[2] + bz, N, log2T, always_hash);
        wgt[q] = (bx ? w[0] : 1.0 - w[0]) * (by ? w[1] : 1.0 - w[1]) * (bz ? w[2] : 1.0 - w[2]);
    }
}

/* feat[n][l*F + f] = sum_c w_c * table[tile][l][idx_c][f]; columns L*F..W-1 are 0.
 * table layout [K][L][T][F] float32.  idx_out (optional) = [n][L][8]. */
void orc_hashgrid_fwd(int L, int F, int log2T, const int32_t *res, int always_hash,
                      const float *table, int64_t n, const float *pos,
                      const uint8_t *tile_id, int W, double *feat, uint32_t *idx_out)
{
    int64_t T = (int64_t)1 << log2T;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        int64_t kt = tile_id ? tile_id[s] : 0;
        double *out = feat + s * W;
        for (int c = 0; c < W; ++c) out[c] = 0.0;
        for (int l = 0; l < L; ++l) {
            uint32_t idx[8];
            double wgt[8];
            orc_hash_corners(pos + 3 * s, res[l], log2T, always_hash, idx, wgt);
            const float *lev = table + ((kt * L + l) * T) * F;
            for (int f = 0; f < F; ++f) {
                double acc = 0.0;
                for (int q = 0; q < 8; ++q) acc += wgt[q] * (double)lev[(int64_t)idx[q] * F + f];
                out[l * F + f] = acc;
            }
            if (idx_out)
                for (int q = 0; q < 8; ++q) idx_out[(s * L + l) * 8 + q] = idx[q];
        }
    }
}

/* dtable[tile][l][idx_c][f] += w_c * dfeat[n][l*F + f]  (FP64 accumulation).
 * Levels own disjoint table slices, so each level is one independent task
 * that visits the samples in order: the result does not depend on threads. */
void orc_hashgrid_bwd(int L, int F, int log2T, const int32_t *res, int always_hash,
                      int K, int64_t n, const float *pos, const uint8_t *tile_id,
                      int W, const double *dfeat, double *dtable)
{
    int64_t T = (int64_t)1 << log2T;
#pragma omp parallel for schedule(dynamic, 1)
    for (int task = 0; task < K * L; ++task) {
        int kt = task / L, l = task % L;
        double *lev = dtable + (((int64_t)kt * L + l) * T) * F;
        for (int64_t s = 0; s < n; ++s) {
            if ((tile_id ? tile_id[s] : 0) != kt) continue;
            uint32_t idx[8];
            double wgt[8];
            orc_hash_corners(pos + 3 * s, res[l], log2T, always_hash, idx, wgt);
            for (int q = 0; q < 8; ++q)
                for (int f = 0; f < F; ++f)
                    lev[(int64_t)idx[q] * F + f] += wgt[q] * dfeat[s * W + l * F + f];
        }
    }
}

/* ------------------------------------------------------------------ */
/* MLP                                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int feat_width, hidden, dens_out, n_dir, colour_layers, colour_out;
} orc_mlp;

static int64_t mlp_offsets(const orc_mlp *m, int64_t off[8])
{
    int cin = m->dens_out - 1 + m->n_dir;
    int64_t o = 0;
    int li = 0;
    off[li++] = o; o += (int64_t)m->hidden * m->feat_width;      /* density L1 */
    off[li++] = o; o += (int64_t)m->dens_out * m->hidden;        /* density L2 */
    off[li++] = o; o += (int64_t)m->hidden * cin;                /* colour L1  */
    for (int c = 1; c < m->colour_layers; ++c) {
        off[li++] = o; o += (int64_t)m->hidden * m->hidden;      /* colour Lc  */
    }
    off[li++] = o; o += (int64_t)m->colour_out * m->hidden;      /* colour out */
    return o;
}

int64_t orc_mlp_param_count(int feat_width, int hidden, int dens_out, int n_dir,
                            int colour_layers, int colour_out)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    return mlp_offsets(&m, off);
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* y = W x for row-major W[out][in] */
static void matvec(const double *W, int out, int in, const double *x, double *y)
{
    for (int o = 0; o < out; ++o) {
        double acc = 0.0;
        for (int i = 0; i < in; ++i) acc += W[(int64_t)o * in + i] * x[i];
        y[o] = acc;
    }
}

#define ORC_MAXW 128
#define ORC_MAX_COLOUR_LAYERS 4

/* Activations of one sample. */
typedef struct {
    double x[ORC_MAXW], h1[ORC_MAXW], o[ORC_MAXW];
    double cin[ORC_MAXW], g[ORC_MAX_COLOUR_LAYERS][ORC_MAXW], out[8];
} orc_act;

static void mlp_forward_one(const orc_mlp *m, const double *w, const int64_t *off,
                            const double *feat, const float *view, const float *sun,
                            orc_act *a, double *sigma, double rgb[3])
{
    int H = m->hidden, cin = m->dens_out - 1 + m->n_dir;
    for (int i = 0; i < m->feat_width; ++i) a->x[i] = feat[i];
    matvec(w + off[0], H, m->feat_width, a->x, a->h1);
    for (int i = 0; i < H; ++i) a->h1[i] = a->h1[i] > 0.0 ? a->h1[i] : 0.0;
    matvec(w + off[1], m->dens_out, H, a->h1, a->o);
    *sigma = exp(a->o[0]);
    for (int i = 0; i < m->dens_out - 1; ++i) a->cin[i] = a->o[1 + i];
    for (int i = 0; i < 3; ++i) a->cin[m->dens_out - 1 + i] = view[i];
    if (m->n_dir == 6)
        for (int i = 0; i < 3; ++i) a->cin[m->dens_out + 2 + i] = sun[i];
    matvec(w + off[2], H, cin, a->cin, a->g[0]);
    for (int i = 0; i < H; ++i) a->g[0][i] = a->g[0][i] > 0.0 ? a->g[0][i] : 0.0;
    for (int c = 1; c < m->colour_layers; ++c) {
        matvec(w + off[2 + c], H, H, a->g[c - 1], a->g[c]);
        for (int i = 0; i < H; ++i) a->g[c][i] = a->g[c][i] > 0.0 ? a->g[c][i] : 0.0;
    }
    matvec(w + off[2 + m->colour_layers], m->colour_out, H, a->g[m->colour_layers - 1], a->out);
    if (m->colour_out == 3) {
        for (int c = 0; c < 3; ++c) rgb[c] = sigmoid(a->out[c]);
    } else { /* albedo rgb times scalar sun visibility */
        double vis = sigmoid(a->out[3]);
        for (int c = 0; c < 3; ++c) rgb[c] = sigmoid(a->out[c]) * vis;
    }
}

/* Distance of one sample from the nearest ReLU kink: the minimum over every
 * hidden pre-activation z of |z| / sum_i |W_i x_i|.  A sample whose margin is
 * below the working precision of an implementation may legitimately get the
 * other ReLU decision there; tests use this to tell ambiguous samples apart. */
static double relu_margin_layer(const double *W, int out, int in, const double *x, double *y)
{
    double m = INFINITY;
    for (int o = 0; o < out; ++o) {
        double acc = 0.0, l1 = 0.0;
        for (int i = 0; i < in; ++i) {
            acc += W[(int64_t)o * in + i] * x[i];
            l1 += fabs(W[(int64_t)o * in + i] * x[i]);
        }
        y[o] = acc;
        if (l1 > 0.0 && fabs(acc) / l1 < m) m = fabs(acc) / l1;
    }
    return m;
}

static double *weights_f64(const float *wf, int64_t P)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)P);
    for (int64_t i = 0; i < P; ++i) w[i] = (double)wf[i];
    return w;
}

/*
 * Density net: h = relu(Wd1 feat); o = Wd2 h; sigma = exp(o_0); emb = o_1.. .
 * Colour net: input [emb, view(3), sun(3) if n_dir == 6]; hidden ReLU layers;
 * rgb = sigmoid(out) (colour_out 3) or sigmoid(out_0..2) * sigmoid(out_3)
 * (colour_out 4).  No biases.  feat is [n][feat_width], view/sun are per ray.
 */
void orc_mlp_fwd(int feat_width, int hidden, int dens_out, int n_dir, int colour_layers,
                 int colour_out, const float *weights, int64_t n, const double *feat,
                 const float *view, const float *sun, const int32_t *ray_id,
                 double *sigma, double *rgb)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    int64_t P = mlp_offsets(&m, off);
    double *w = weights_f64(weights, P);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        orc_act a;
        int64_t r = ray_id[s];
        mlp_forward_one(&m, w, off, feat + s * feat_width, view + 3 * r,
                        sun ? sun + 3 * r : NULL, &a, sigma + s, rgb + 3 * s);
    }
    free(w);
}

/* Per-sample ReLU margin (see relu_margin_layer) of the forward pass. */
void orc_mlp_margin(int feat_width, int hidden, int dens_out, int n_dir, int colour_layers,
                    int colour_out, const float *weights, int64_t n, const double *feat,
                    const float *view, const float *sun, const int32_t *ray_id, double *margin)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    int64_t P = mlp_offsets(&m, off);
    double *w = weights_f64(weights, P);
    int H = hidden, cin = dens_out - 1 + n_dir;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        orc_act a;
        int64_t r = ray_id[s];
        double sig, rgb[3];
        mlp_forward_one(&m, w, off, feat + s * feat_width, view + 3 * r, sun ? sun + 3 * r : NULL,
                        &a, &sig, rgb);
        double y[ORC_MAXW];
        double mg = relu_margin_layer(w + off[0], H, feat_width, a.x, y);
        double t = relu_margin_layer(w + off[2], H, cin, a.cin, y);
        if (t < mg) mg = t;
        for (int c = 1; c < colour_layers; ++c) {
            t = relu_margin_layer(w + off[2 + c], H, H, a.g[c - 1], y);
            if (t < mg) mg = t;
        }
        margin[s] = mg;
    }
    free(w);
}

/* Forward with BF16 rounding emulated at the points where a BF16 matrix-core
 * implementation rounds: features, weights, the embedding and directions fed
 * to the colour net, and every post-ReLU hidden activation are rounded to the
 * nearest bfloat16 (ties to even, via float32); sums stay exact in FP64;
 * sigma = exp(o_0) uses the unrounded logit.  Diagnostic only. */
static double bf16r(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) {
        u += 0x7fffu + ((u >> 16) & 1u);
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

/* out[i] = in[i] rounded to the nearest bfloat16 (ties to even, via float32). */
void orc_bf16_round(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16r(in[i]);
}

void orc_mlp_fwd_bf16emu(int feat_width, int hidden, int dens_out, int n_dir, int colour_layers,
                         int colour_out, const float *weights, int64_t n, const double *feat,
                         const float *view, const float *sun, const int32_t *ray_id,
                         double *sigma, double *rgb)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    int64_t P = mlp_offsets(&m, off);
    double *w = weights_f64(weights, P);
    for (int64_t i = 0; i < P; ++i) w[i] = bf16r(w[i]);
    int H = hidden, cin = dens_out - 1 + n_dir, CL = colour_layers;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double x[ORC_MAXW] = {0}, h[ORC_MAXW] = {0}, o[ORC_MAXW] = {0}, ci[ORC_MAXW] = {0};
        double g[ORC_MAXW] = {0}, g2[ORC_MAXW] = {0}, out[8] = {0};
        int64_t r = ray_id[s];
        for (int i = 0; i < feat_width; ++i) x[i] = bf16r(feat[s * feat_width + i]);
        matvec(w + off[0], H, feat_width, x, h);
        for (int i = 0; i < H; ++i) h[i] = bf16r(h[i] > 0.0 ? h[i] : 0.0);
        matvec(w + off[1], dens_out, H, h, o);
        sigma[s] = exp(o[0]);
        for (int i = 0; i < dens_out - 1; ++i) ci[i] = bf16r(o[1 + i]);
        for (int i = 0; i < 3; ++i) ci[dens_out - 1 + i] = bf16r(view[3 * r + i]);
        if (n_dir == 6)
            for (int i = 0; i < 3; ++i) ci[dens_out + 2 + i] = bf16r(sun[3 * r + i]);
        matvec(w + off[2], H, cin, ci, g);
        for (int i = 0; i < H; ++i) g[i] = bf16r(g[i] > 0.0 ? g[i] : 0.0);
        for (int c = 1; c < CL; ++c) {
            matvec(w + off[2 + c], H, H, g, g2);
            for (int i = 0; i < H; ++i) g[i] = bf16r(g2[i] > 0.0 ? g2[i] : 0.0);
        }
        matvec(w + off[2 + CL], colour_out, H, g, out);
        if (colour_out == 3) {
            for (int c = 0; c < 3; ++c) rgb[3 * s + c] = sigmoid(out[c]);
        } else {
            double vis = sigmoid(out[3]);
            for (int c = 0; c < 3; ++c) rgb[3 * s + c] = sigmoid(out[c]) * vis;
        }
    }
    free(w);
}

/* Adjoint of one sample: forward again, then back through every layer.
 * Adds this sample's outer products into dw (packed like the weights) and
 * writes d(loss)/d(feat) into dfeat. */
static void mlp_adjoint_one(const orc_mlp *m, const double *w, const int64_t *off,
                            const double *feat, const float *view, const float *sun,
                            double dsigma, const double drgb[3], double *dw, double *dfeat)
{
    int H = m->hidden, cin = m->dens_out - 1 + m->n_dir, CL = m->colour_layers;
    int FW = m->feat_width, DO = m->dens_out, CO = m->colour_out;
    orc_act a;
    double sig, rgb[3];
    mlp_forward_one(m, w, off, feat, view, sun, &a, &sig, rgb);

    /* output activation */
    double dout[8];
    if (CO == 3) {
        for (int c = 0; c < 3; ++c) {
            double y = sigmoid(a.out[c]);
            dout[c] = drgb[c] * y * (1.0 - y);
        }
    } else {
        double vis = sigmoid(a.out[3]), dvis = 0.0;
        for (int c = 0; c < 3; ++c) {
            double alb = sigmoid(a.out[c]);
            dout[c] = drgb[c] * vis * alb * (1.0 - alb);
            dvis += drgb[c] * alb;
        }
        dout[3] = dvis * vis * (1.0 - vis);
    }

    /* colour output layer: W[CO][H] applied to g[CL-1] */
    double dg[ORC_MAXW], tmp[ORC_MAXW];
    {
        const double *W = w + off[2 + CL];
        double *dW = dw + off[2 + CL];
        const double *x = a.g[CL - 1];
        for (int o = 0; o < CO; ++o)
            for (int i = 0; i < H; ++i) dW[(int64_t)o * H + i] += dout[o] * x[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < CO; ++o) acc += W[(int64_t)o * H + i] * dout[o];
            dg[i] = x[i] > 0.0 ? acc : 0.0;          /* through the ReLU of g[CL-1] */
        }
    }
    /* colour hidden layers c = CL-1 .. 1: W[H][H] applied to g[c-1] */
    for (int c = CL - 1; c >= 1; --c) {
        const double *W = w + off[2 + c];
        double *dW = dw + off[2 + c];
        const double *x = a.g[c - 1];
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < H; ++i) dW[(int64_t)o * H + i] += dg[o] * x[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += W[(int64_t)o * H + i] * dg[o];
            tmp[i] = x[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < H; ++i) dg[i] = tmp[i];
    }
    /* colour first layer: W[H][cin] applied to cin = [emb, view, sun] */
    double dos[ORC_MAXW];
    {
        const double *W = w + off[2];
        double *dW = dw + off[2];
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < cin; ++i) dW[(int64_t)o * cin + i] += dg[o] * a.cin[i];
        dos[0] = dsigma * exp(a.o[0]);               /* sigma = exp(o_0) */
        for (int e = 0; e < DO - 1; ++e) {          /* emb = o_1.. (directions get no gradient) */
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += W[(int64_t)o * cin + e] * dg[o];
            dos[1 + e] = acc;
        }
    }
    /* density second layer: W[DO][H] applied to h1 */
    double dh[ORC_MAXW];
    {
        const double *W = w + off[1];
        double *dW = dw + off[1];
        for (int o = 0; o < DO; ++o)
            for (int i = 0; i < H; ++i) dW[(int64_t)o * H + i] += dos[o] * a.h1[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < DO; ++o) acc += W[(int64_t)o * H + i] * dos[o];
            dh[i] = a.h1[i] > 0.0 ? acc : 0.0;
        }
    }
    /* density first layer: W[H][FW] applied to feat */
    {
        const double *W = w + off[0];
        double *dW = dw + off[0];
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < FW; ++i) dW[(int64_t)o * FW + i] += dh[o] * a.x[i];
        for (int i = 0; i < FW; ++i) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += W[(int64_t)o * FW + i] * dh[o];
            dfeat[i] = acc;
        }
    }
}

/* q16(x, on): x rounded to the nearest bfloat16 when `on`, else x. */
static double q16(double x, int on) { return on ? bf16r(x) : x; }

/* Adjoint of one sample with every matrix-core operand of a 16-bit
 * implementation rounded to bfloat16 (when q): the weights, the network
 * inputs, the post-ReLU activations and colour inputs (as in the forward
 * emulation above), and in the adjoint the output gradient fed to each
 * transposed product and both factors of every weight-gradient outer product.
 * ReLU masks, sigmoid and exp use the unrounded values; sums are FP64.  With
 * q == 0 it is the plain FP64 adjoint, term for term in the same order as
 * mlp_adjoint_one (w must already hold rounded weights when q != 0). */
static void mlp_adjoint_one_q(const orc_mlp *m, const double *w, const int64_t *off,
                              const double *feat, const float *view, const float *sun,
                              double dsigma, const double drgb[3], double *dw, double *dfeat, int q)
{
    int H = m->hidden, cin = m->dens_out - 1 + m->n_dir, CL = m->colour_layers;
    int FW = m->feat_width, DO = m->dens_out, CO = m->colour_out;
    /* forward with the operands rounded where a 16-bit matrix core takes them */
    double x[ORC_MAXW], h1[ORC_MAXW], o[ORC_MAXW], ci[ORC_MAXW], g[ORC_MAX_COLOUR_LAYERS][ORC_MAXW];
    double out[8];
    for (int i = 0; i < FW; ++i) x[i] = q16(feat[i], q);
    matvec(w + off[0], H, FW, x, h1);
    for (int i = 0; i < H; ++i) h1[i] = h1[i] > 0.0 ? h1[i] : 0.0;
    double h1q[ORC_MAXW];
    for (int i = 0; i < H; ++i) h1q[i] = q16(h1[i], q);
    matvec(w + off[1], DO, H, h1q, o);
    for (int i = 0; i < DO - 1; ++i) ci[i] = q16(o[1 + i], q);
    for (int i = 0; i < 3; ++i) ci[DO - 1 + i] = q16(view[i], q);
    if (m->n_dir == 6)
        for (int i = 0; i < 3; ++i) ci[DO + 2 + i] = q16(sun[i], q);
    double gq[ORC_MAX_COLOUR_LAYERS][ORC_MAXW];
    matvec(w + off[2], H, cin, ci, g[0]);
    for (int i = 0; i < H; ++i) {
        g[0][i] = g[0][i] > 0.0 ? g[0][i] : 0.0;
        gq[0][i] = q16(g[0][i], q);
    }
    for (int c = 1; c < CL; ++c) {
        matvec(w + off[2 + c], H, H, gq[c - 1], g[c]);
        for (int i = 0; i < H; ++i) {
            g[c][i] = g[c][i] > 0.0 ? g[c][i] : 0.0;
            gq[c][i] = q16(g[c][i], q);
        }
    }
    matvec(w + off[2 + CL], CO, H, gq[CL - 1], out);

    /* output activation */
    double dout[8];
    if (CO == 3) {
        for (int c = 0; c < 3; ++c) {
            double y = sigmoid(out[c]);
            dout[c] = drgb[c] * y * (1.0 - y);
        }
    } else {
        double vis = sigmoid(out[3]), dvis = 0.0;
        for (int c = 0; c < 3; ++c) {
            double alb = sigmoid(out[c]);
            dout[c] = drgb[c] * vis * alb * (1.0 - alb);
            dvis += drgb[c] * alb;
        }
        dout[3] = dvis * vis * (1.0 - vis);
    }
    for (int c = 0; c < CO; ++c) dout[c] = q16(dout[c], q);

    /* colour output layer */
    double dg[ORC_MAXW], tmp[ORC_MAXW];
    {
        const double *W = w + off[2 + CL];
        double *dW = dw + off[2 + CL];
        const double *xi = gq[CL - 1];
        for (int oo = 0; oo < CO; ++oo)
            for (int i = 0; i < H; ++i) dW[(int64_t)oo * H + i] += dout[oo] * xi[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int oo = 0; oo < CO; ++oo) acc += W[(int64_t)oo * H + i] * dout[oo];
            dg[i] = g[CL - 1][i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < H; ++i) dg[i] = q16(dg[i], q);
    }
    /* colour hidden layers */
    for (int c = CL - 1; c >= 1; --c) {
        const double *W = w + off[2 + c];
        double *dW = dw + off[2 + c];
        const double *xi = gq[c - 1];
        for (int oo = 0; oo < H; ++oo)
            for (int i = 0; i < H; ++i) dW[(int64_t)oo * H + i] += dg[oo] * xi[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int oo = 0; oo < H; ++oo) acc += W[(int64_t)oo * H + i] * dg[oo];
            tmp[i] = g[c - 1][i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < H; ++i) dg[i] = q16(tmp[i], q);
    }
    /* colour first layer */
    double dos[ORC_MAXW];
    {
        const double *W = w + off[2];
        double *dW = dw + off[2];
        for (int oo = 0; oo < H; ++oo)
            for (int i = 0; i < cin; ++i) dW[(int64_t)oo * cin + i] += dg[oo] * ci[i];
        dos[0] = dsigma * exp(o[0]);
        for (int e = 0; e < DO - 1; ++e) {
            double acc = 0.0;
            for (int oo = 0; oo < H; ++oo) acc += W[(int64_t)oo * cin + e] * dg[oo];
            dos[1 + e] = acc;
        }
        for (int e = 0; e < DO; ++e) dos[e] = q16(dos[e], q);
    }
    /* density second layer */
    double dh[ORC_MAXW];
    {
        const double *W = w + off[1];
        double *dW = dw + off[1];
        for (int oo = 0; oo < DO; ++oo)
            for (int i = 0; i < H; ++i) dW[(int64_t)oo * H + i] += dos[oo] * h1q[i];
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int oo = 0; oo < DO; ++oo) acc += W[(int64_t)oo * H + i] * dos[oo];
            dh[i] = h1[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < H; ++i) dh[i] = q16(dh[i], q);
    }
    /* density first layer */
    {
        const double *W = w + off[0];
        double *dW = dw + off[0];
        for (int oo = 0; oo < H; ++oo)
            for (int i = 0; i < FW; ++i) dW[(int64_t)oo * FW + i] += dh[oo] * x[i];
        for (int i = 0; i < FW; ++i) {
            double acc = 0.0;
            for (int oo = 0; oo < H; ++oo) acc += W[(int64_t)oo * FW + i] * dh[oo];
            dfeat[i] = acc;
        }
    }
}

#define ORC_CHUNKS 64

/* Adjoint of orc_mlp_fwd.  dW (packed like the weights) is ADDED TO; dfeat
 * [n][feat_width] is written.  Samples are split into ORC_CHUNKS fixed
 * contiguous chunks whose partial sums are added in chunk order, so the
 * result does not depend on the number of threads. */
void orc_mlp_bwd(int feat_width, int hidden, int dens_out, int n_dir, int colour_layers,
                 int colour_out, const float *weights, int64_t n, const double *feat,
                 const float *view, const float *sun, const int32_t *ray_id,
                 const double *dsigma, const double *drgb, double *dW, double *dfeat)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    int64_t P = mlp_offsets(&m, off);
    double *w = weights_f64(weights, P);
    double *part = (double *)calloc((size_t)ORC_CHUNKS * (size_t)P, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        int64_t s0 = n * ch / ORC_CHUNKS, s1 = n * (ch + 1) / ORC_CHUNKS;
        for (int64_t s = s0; s < s1; ++s) {
            int64_t r = ray_id[s];
            mlp_adjoint_one(&m, w, off, feat + s * feat_width, view + 3 * r,
                            sun ? sun + 3 * r : NULL, dsigma[s], drgb + 3 * s,
                            part + (int64_t)ch * P, dfeat + s * feat_width);
        }
    }
    for (int ch = 0; ch < ORC_CHUNKS; ++ch)
        for (int64_t i = 0; i < P; ++i) dW[i] += part[(int64_t)ch * P + i];
    free(part);
    free(w);
}

/* Adjoint of the 16-bit form: orc_mlp_bwd with every matrix-core operand
 * rounded to bfloat16 (mlp_adjoint_one_q, q = round16); round16 == 0 gives
 * the plain FP64 adjoint again, bit for bit equal to orc_mlp_bwd.  Same
 * chunked, thread-count independent summation of dW. */
void orc_mlp_bwd_q(int feat_width, int hidden, int dens_out, int n_dir, int colour_layers,
                   int colour_out, const float *weights, int64_t n, const double *feat,
                   const float *view, const float *sun, const int32_t *ray_id,
                   const double *dsigma, const double *drgb, int round16, double *dW, double *dfeat)
{
    orc_mlp m = {feat_width, hidden, dens_out, n_dir, colour_layers, colour_out};
    int64_t off[8];
    int64_t P = mlp_offsets(&m, off);
    double *w = weights_f64(weights, P);
    for (int64_t i = 0; i < P; ++i) w[i] = q16(w[i], round16);
    double *part = (double *)calloc((size_t)ORC_CHUNKS * (size_t)P, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        int64_t s0 = n * ch / ORC_CHUNKS, s1 = n * (ch + 1) / ORC_CHUNKS;
        for (int64_t s = s0; s < s1; ++s) {
            int64_t r = ray_id[s];
            mlp_adjoint_one_q(&m, w, off, feat + s * feat_width, view + 3 * r,
                              sun ? sun + 3 * r : NULL, dsigma[s], drgb + 3 * s,
                              part + (int64_t)ch * P, dfeat + s * feat_width, round16);
        }
    }
    for (int ch = 0; ch < ORC_CHUNKS; ++ch)
        for (int64_t i = 0; i < P; ++i) dW[i] += part[(int64_t)ch * P + i];
    free(part);
    free(w);
}

/* ------------------------------------------------------------------ */
/* Volume rendering and loss                                           */
/* ------------------------------------------------------------------ */

/*
 * Per ray r over its samples i (packed_info[r] = (start, count)):
 *   delta_i = t1_i - t0_i, s_i = sigma_i delta_i,
 *   T_i = exp(-sum_{j<i} s_j), alpha_i = 1 - exp(-s_i), w_i = T_i alpha_i,
 *   C = sum w_i c_i, opacity = sum w_i, depth = sum w_i (t0_i + t1_i)/2,
 * background 0.  With early_stop_T > 0 only the samples with T_i >= early_stop_T
 * are kept (a prefix, since T is non-increasing); n_alive[r] is their count.
 * If alive_in is given it fixes the kept count instead.
 * loss = loss_scale * sum_r sum_ch (C - target)^2 when target is given.
 */
void orc_composite_fwd(int R, const int32_t *packed_info, const double *sigma,
                       const double *rgb, const float *t0, const float *t1,
                       double early_stop_T, const int32_t *alive_in,
                       const float *target, double loss_scale,
                       double *rgb_out, double *opacity, double *depth,
                       int32_t *n_alive, double *loss)
{
    double total = 0.0;
    for (int r = 0; r < R; ++r) {
        int64_t st = packed_info[2 * r], cnt = packed_info[2 * r + 1];
        double C[3] = {0, 0, 0}, acc = 0.0, dep = 0.0, tau = 0.0;
        int64_t kept = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            int64_t s = st + i;
            double T = exp(-tau);
            if (alive_in) {
                if (i >= alive_in[r]) break;
            } else if (early_stop_T > 0.0 && T < early_stop_T) {
                break;
            }
            double delta = (double)t1[s] - (double)t0[s];
            double si = sigma[s] * delta;
            double w = T * (1.0 - exp(-si));
            for (int c = 0; c < 3; ++c) C[c] += w * rgb[3 * s + c];
            acc += w;
            dep += w * 0.5 * ((double)t0[s] + (double)t1[s]);
            tau += si;
            ++kept;
        }
        for (int c = 0; c < 3; ++c) rgb_out[3 * r + c] = C[c];
        if (opacity) opacity[r] = acc;
        if (depth) depth[r] = dep;
        if (n_alive) n_alive[r] = (int32_t)kept;
        if (target)
            for (int c = 0; c < 3; ++c) {
                double e = C[c] - (double)target[3 * r + c];
                total += e * e;
            }
    }
    if (loss) *loss = loss_scale * total;
}

/*
 * Adjoint of the composite for the loss above, g = dL/dC = 2 loss_scale (C - target):
 *   dL/dc_i     = w_i g,
 *   dL/dsigma_i = delta_i sum_ch g_ch (T_{i+1} c_i,ch - (C_ch - A_i,ch)),
 * with A_i = sum_{j<=i} w_j c_j.  Samples past n_alive[r] get zero gradient.
 */
void orc_composite_bwd(int R, const int32_t *packed_info, const double *sigma,
                       const double *rgb, const float *t0, const float *t1,
                       const int32_t *n_alive, const float *target, double loss_scale,
                       double *dsigma, double *drgb)
{
    for (int r = 0; r < R; ++r) {
        int64_t st = packed_info[2 * r], cnt = packed_info[2 * r + 1];
        int64_t kept = n_alive ? n_alive[r] : cnt;
        /* forward again to get C */
        double C[3] = {0, 0, 0}, tau = 0.0;
        for (int64_t i = 0; i < kept; ++i) {
            int64_t s = st + i;
            double delta = (double)t1[s] - (double)t0[s];
            double si = sigma[s] * delta;
            double w = exp(-tau) * (1.0 - exp(-si));
            for (int c = 0; c < 3; ++c) C[c] += w * rgb[3 * s + c];
            tau += si;
        }
        double g[3];
        for (int c = 0; c < 3; ++c) g[c] = 2.0 * loss_scale * (C[c] - (double)target[3 * r + c]);
        double A[3] = {0, 0, 0};
        tau = 0.0;
        for (int64_t i = 0; i < cnt; ++i) {
            int64_t s = st + i;
            if (i >= kept) {
                dsigma[s] = 0.0;
                for (int c = 0; c < 3; ++c) drgb[3 * s + c] = 0.0;
                continue;
            }
            double delta = (double)t1[s] - (double)t0[s];
            double si = sigma[s] * delta;
            double T = exp(-tau);
            double w = T * (1.0 - exp(-si));
            double Tn = exp(-(tau + si));
            double ds = 0.0;
            for (int c = 0; c < 3; ++c) {
                A[c] += w * rgb[3 * s + c];
                drgb[3 * s + c] = w * g[c];
                ds += g[c] * (Tn * rgb[3 * s + c] - (C[c] - A[c]));
            }
            dsigma[s] = delta * ds;
            tau += si;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Adam                                                                */
/* ------------------------------------------------------------------ */

/* One Adam step (bias-corrected), step = t >= 1, in FP64 on FP64 state:
 *   g' = g + l2 p; m = b1 m + (1-b1) g'; v = b2 v + (1-b2) g'^2;
 *   p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_adam_step(int64_t n, double *p, const double *g, double *m, double *v,
                   double lr, double b1, double b2, double eps, int step, double l2)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        double gi = g[i] + l2 * p[i];
        m[i] = b1 * m[i] + (1.0 - b1) * gi;
        v[i] = b2 * v[i] + (1.0 - b2) * gi * gi;
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
