/*
 * libsnake -- one training step of a tile NeRF on AMD Instinct MI355X (gfx950).
 *
 * Method: "Tile and Slide: A New Framework for Scaling NeRF from Local to
 * Global 3D Earth Observation" (Snake-NeRF, arXiv 2507.01631).  A large scene
 * is cut into non-overlapping NeRF tiles (Sec. 4.2); each NeRF is a
 * multiresolution hash encoding feeding a local density network whose
 * embedding feeds a colour network (Sec. 4.1); rays are cut at tile
 * boundaries and sampled per segment (Sec. 4.5); colours come from the
 * unmodified volume-rendering quadrature and a colour-consistency loss
 * (Sec. 2.2, 4.4); optimisation follows the I-NGP strategy (Sec. 4.6).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *     row-major, aligned to their element size (16 B for float4-read arrays
 *     where stated).  Scalars and descriptor structs are host values.
 *   - The library allocates nothing in these calls; scratch memory is the
 *     caller's `workspace`, sized by the matching *_workspace_bytes query.
 *   - Every call is asynchronous on the HIP stream passed last (0 = the null
 *     stream) and returns a snake_status.  Argument errors are detected on the
 *     host before any launch and leave outputs untouched; the message is
 *     available from snake_last_error() (thread-local).
 *   - Sample counts may live on the device: where a call takes `n` (host, an
 *     upper bound used to size the launch) and `n_dev` (device int64, may be
 *     NULL), the effective count is min(n, *n_dev).  No call synchronises the
 *     host, so a step can be captured in a HIP graph.
 *   - Gradient outputs ACCUMULATE (+=); the caller zeroes them.
 *   - Sample-indexed inputs may be read through an optional index list
 *     `sample_idx` (device int32, NULL = identity): entry j of the call reads
 *     input sample sample_idx[j] and writes its per-sample outputs at j.
 *
 * Data layouts
 *   rays        rays_o, rays_d  [R][3] double, world frame (e.g. UTM metres)
 *   NeRF tiles  boxes [K][6] double: lo_x lo_y lo_z hi_x hi_y hi_z
 *   samples     packed per ray, t-ordered: packed_info [R][2] int32 (start,
 *               count); t0, t1 [N] float (world ray parameter); pos [N][3]
 *               float in the tile's [0,1]^3 frame; ray_id [N] int32;
 *               tile_id [N] uint8
 *   table       [K][L][T][F] float (T = 2^log2_table entries per level)
 *   features    level-major [L][N][F] (float, or bf16 when requested), so
 *               that every level reads and writes coalesced; the level
 *               stride is the call's host bound `n` unless stated
 *   MLP weights one float vector, row-major [out][in] matrices packed in the
 *               order of snake_mlp_param_count()
 */
#ifndef SNAKE_H
#define SNAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNAKE_ABI_VERSION 1

typedef struct ihipStream_t *snake_stream_t;   /* == hipStream_t */

typedef enum {
    SNAKE_OK = 0,
    SNAKE_ERR_INVALID_ARG = -1,   /* a size, count or descriptor field is out of range */
    SNAKE_ERR_NULL = -2,          /* a required pointer is NULL */
    SNAKE_ERR_ALIGN = -3,         /* a pointer is not aligned as documented */
    SNAKE_ERR_UNSUPPORTED = -4,   /* valid but not implemented (e.g. F not in {1,2,4}) */
    SNAKE_ERR_HIP = -5,           /* a HIP runtime call failed (launch error) */
    SNAKE_ERR_WORKSPACE = -6,     /* workspace NULL or smaller than required */
    SNAKE_ERR_DEVICE = -7         /* snake_check_device_error found a device-side error */
} snake_status;

/* Device-side error bits, reported by snake_check_device_error(). */
#define SNAKE_DEVERR_CAPACITY 1u  /* sampler: packed samples exceed `cap` */
#define SNAKE_DEVERR_TILE_ID 2u   /* a tile_id >= K (the sample is dropped) */
#define SNAKE_DEVERR_RAY_ID 4u    /* a ray_id >= R (the sample is dropped) */
#define SNAKE_DEVERR_INTERNAL 8u  /* an internal consistency check failed (nothing written out of range) */
#define SNAKE_DEVERR_NONFINITE 16u /* binned table adjoint: a non-finite feature gradient (its level adds nothing) */

typedef enum { SNAKE_F32 = 0, SNAKE_BF16 = 1 } snake_dtype;

/* Library version (SNAKE_ABI_VERSION). */
int snake_abi_version(void);

/* A stream of default priority on a hardware queue of its own (a CU-masked
 * queue with every compute unit enabled): streams created the usual way share
 * a small pool of hardware queues, and two streams on one queue run their
 * work one after the other, so the host transfers of a tile swap would wait
 * for the training they should overlap.  *stream receives the handle; the
 * caller releases it with snake_stream_destroy once no pending work or
 * framework bookkeeping (events recorded at a later free) refers to it. */
int snake_stream_create_dedicated(snake_stream_t *stream);
int snake_stream_destroy(snake_stream_t stream);

/* Message of the last failing call on this thread ("" if none). */
const char *snake_last_error(void);

/* Synchronises `stream`, then reads and clears the device error word of the
 * current device.  Returns SNAKE_OK, or SNAKE_ERR_DEVICE with the error bits
 * in *bits (may be NULL). */
int snake_check_device_error(snake_stream_t stream, uint32_t *bits);

/*
 * Launch-shape tunables.  The process-wide table below is the library's only
 * global state; an autotuner times the calls it affects and sets it before a
 * step is captured (a captured graph keeps the shapes it was captured with).
 * Every value only changes how work is split across the chip, never a
 * result, except where noted.  snake_tune_set returns SNAKE_ERR_INVALID_ARG
 * for an unknown id or a value outside the stated range; 0 restores the
 * default where a default is listed as 0.
 */
typedef enum {
    SNAKE_TUNE_HASH_FWD_BLOCKS_PER_CU = 0,  /* hash-grid forward grid, 1..64 (16) */
    SNAKE_TUNE_MLP_FWD_BLOCKS_PER_CU = 1,   /* network forward grid, 1..16 (8) */
    SNAKE_TUNE_MLP_BWD_BLOCKS_PER_CU = 2,   /* network adjoint grid, 0..2 (0: 2 for BF16,
                                               1 for FP32); changes the dW summation order */
    SNAKE_TUNE_COMPOSITE_BLOCKS_PER_CU = 3, /* rendering grid, 1..64 (8) */
    SNAKE_TUNE_BIN_BLOCKS = 4,              /* binned table adjoint: count/scatter blocks,
                                               64..2048 (2048) */
    SNAKE_TUNE_BIN_LEVELS_PER_PASS = 5,     /* binned table adjoint: most levels per pass,
                                               0..32 (0: as many as the workspace holds) */
    SNAKE_TUNE_SAMPLER_BLOCKS_PER_CU = 6,   /* sampler fill grid, 1..64 (16) */
    SNAKE_TUNE_HASH_FWD_SUPERCHUNK = 7,     /* hash-grid forward work order, 0..64 (0): 0 walks
                                               level by level over all samples; v > 0 walks
                                               super-chunks of v x 2^20 samples, every level of
                                               one before the next (their positions then stay
                                               in the on-package cache across levels) */
    SNAKE_TUNE_HASH_FWD_LDS = 8,            /* hash-grid forward, 0..1 (1): 1 gathers every level
                                               whose slice of one tile fits in a block's LDS from
                                               an LDS copy of it, 0 gathers all levels through
                                               the caches (same results either way) */
    SNAKE_TUNE_COUNT = 9
} snake_tunable;

int snake_tune_set(int32_t which, int32_t value);
int32_t snake_tune_get(int32_t which);   /* -1 for an unknown id */

/* ------------------------------------------------------------------------ */
/* Segmented sampler (Sec. 4.5 with the distribution kernel of Sec. 4.6 and  */
/* the UTM-to-local mapping of Sec. 4.1-4.2)                                 */
/* ------------------------------------------------------------------------ */

/*
 * For each ray, intersect it in FP64 with each of the K NeRF-tile boxes
 * (optionally clipped in z to the altitude band zband = [z_lo, z_hi], host
 * pointer or NULL), sort the hit segments by entry distance, and give the
 * ray's budget S_r = samples_per_ray ? samples_per_ray[r] : S samples to its
 * segments: one each when S_r >= #segments, the rest in proportion to
 * segment length by cumulative rounding (rint(E * cum/total)), so that
 * the counts sum to S_r.  max_count (device, NULL = none) truncates ray r to
 * its first max_count[r] samples (early stop); the kept samples are bit for
 * bit the prefix of the untruncated ones.
 *
 * A segment [t_near, t_far] with n samples gives the intervals
 * [t_j, t_{j+1}]: tn = fl32(t_near), tf = fl32(t_far),
 * step = fl32(fl32(tf - tn)/n), t_j = fl32(tn + fl32(j*step)), t_n = tf.
 * Each interval is evaluated at its midpoint m = fl32(0.5 fl32(t_j+t_{j+1}))
 * mapped to the tile's frame: pos_a = clamp(fl32(o'_a + fl32(m d'_a)), 0, 1)
 * with o'_a = fl32((o_a-lo_a)/(hi_a-lo_a)), d'_a = fl32(d_a/(hi_a-lo_a)).
 * A slab hit needs t_far > t_near (t_near clamped at 0); an axis-parallel
 * ray is inside a slab when lo <= o < hi.  Segments of neighbouring tiles
 * meet bit-exactly on their shared face.  view[R][3] = fl32(d/|d|).
 *
 * Outputs: packed_info [R][2]; t0, t1, pos, ray_id, tile_id (tile_id may be
 * NULL when K == 1) for up to `cap` samples; *n_out (device int64) = the
 * packed total.  If the total exceeds cap, samples past cap are not written
 * and SNAKE_DEVERR_CAPACITY is raised on the device.
 * boxes [K][6] and zband [2] are HOST pointers, copied at call time.
 * Workspace: snake_sample_workspace_bytes(R).  Limits: 1 <= K <= 16.
 */
size_t snake_sample_workspace_bytes(int32_t R);
int snake_sample_segmented(const double *rays_o, const double *rays_d, int32_t R,
                           const double *boxes, int32_t K, const double *zband,
                           const int32_t *samples_per_ray, int32_t S,
                           const int32_t *max_count,
                           int32_t *packed_info, float *t0, float *t1, float *pos,
                           int32_t *ray_id, uint8_t *tile_id, float *view,
                           int64_t cap, int64_t *n_out,
                           void *workspace, size_t workspace_bytes, snake_stream_t stream);

/*
 * The sampler with its samples grouped by tile, for the window step (Sec.
 * 4.4), where each loaded tile has its own networks: the same samples as
 * snake_sample_segmented with the same arguments, and packed_info [R][2],
 * t0, t1 and view as there (packed, ray by ray), but pos [][3], ray_id and
 * tile_id (not NULL) written tile by tile, ray by ray within a tile, in t
 * within a ray -- the order snake_tile_partition gives the packed samples.
 * sample_map [n] int32 (device) maps a packed index to its grouped index
 * (that partition's inv), and tile_start [K+2] int64 (device) bounds the
 * groups: tile k holds grouped indices tile_start[k] .. tile_start[k+1]-1,
 * and tile_start[K] = tile_start[K+1] = *n_out.  Replaces the sampler and
 * the partition with one count, two scans and one fill.  R * K < 2^31.
 * When the total exceeds cap (SNAKE_DEVERR_CAPACITY), a sample whose grouped
 * index would be cap or more is not written and its sample_map entry is
 * cap - 1, so that no consumer of the map reads past the arrays.
 * Workspace: snake_sample_grouped_workspace_bytes(R, K) (0 for bad R, K),
 * 256-byte aligned.  Errors as snake_sample_segmented.
 */
size_t snake_sample_grouped_workspace_bytes(int32_t R, int32_t K);
int snake_sample_grouped(const double *rays_o, const double *rays_d, int32_t R,
                         const double *boxes, int32_t K, const double *zband,
                         const int32_t *samples_per_ray, int32_t S, const int32_t *max_count,
                         int32_t *packed_info, float *t0, float *t1, float *view,
                         float *pos, int32_t *ray_id, uint8_t *tile_id, int32_t *sample_map,
                         int64_t *tile_start, int64_t cap, int64_t *n_out,
                         void *workspace, size_t workspace_bytes, snake_stream_t stream);

/*
 * No-allocation variant of snake_sample_segmented, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and results, without the
 * workspace: the count/scan scratch is a static device array of the library
 * sized for R <= snake_sample_segmented_static_max_rays() (2^20 rays, about
 * 8 MiB, held by every device the library runs on until the process ends).
 * A larger R returns SNAKE_ERR_INVALID_ARG before any launch.  The call
 * allocates nothing.  All calls on one device share that device's scratch,
 * so calls that overlap on one device (two streams, two host threads) race:
 * the caller serialises them.  Every call writes all the scratch it reads,
 * so nothing carries over from the previous call.
 */
int32_t snake_sample_segmented_static_max_rays(void);
int snake_sample_segmented_static(const double *rays_o, const double *rays_d, int32_t R,
                                  const double *boxes, int32_t K, const double *zband,
                                  const int32_t *samples_per_ray, int32_t S,
                                  const int32_t *max_count,
                                  int32_t *packed_info, float *t0, float *t1, float *pos,
                                  int32_t *ray_id, uint8_t *tile_id, float *view,
                                  int64_t cap, int64_t *n_out, snake_stream_t stream);

/*
 * Index list of the samples kept by early stop: for each ray r, the first
 * n_alive[r] of its packed samples, in order.  idx_out [cap] int32 receives
 * their packed indices and *n_out (device int64) their total.  Workspace:
 * snake_sample_workspace_bytes(R).
 */
int snake_pack_alive(const int32_t *packed_info, const int32_t *n_alive, int32_t R,
                     int32_t *idx_out, int64_t cap, int64_t *n_out,
                     void *workspace, size_t workspace_bytes, snake_stream_t stream);

/*
 * Ray acceptance of the 2x2 sliding window (Sec. 4.4): while a window of
 * NeRF tiles is loaded, only rays that cross no other tile are trained on.
 * The window's tiles share the altitude band zband = [z_lo, z_hi] and cover
 * the rectangle window = [x_lo, y_lo, x_hi, y_hi] (both HOST pointers,
 * copied at call time).  Ray r is accepted when its chord through the band
 * (t >= 0) is non-empty and bounded (d_z != 0) and both chord end points
 * o + t d have x, y inside the closed rectangle; FP64, no FMA contraction.
 * Outputs: accept [R] uint8 (may be NULL), idx_out [R] int32 = the accepted
 * ray indices in increasing order, *n_out (device int64) = their count.
 * Workspace: snake_sample_workspace_bytes(R).
 */
int snake_window_accept(const double *rays_o, const double *rays_d, int32_t R,
                        const double *window, const double *zband, uint8_t *accept,
                        int32_t *idx_out, int64_t *n_out,
                        void *workspace, size_t workspace_bytes, snake_stream_t stream);

/*
 * Stable partition of n samples by NeRF tile, for the window step where each
 * loaded tile has its own networks (Sec. 4.4): perm [n] int32 lists the
 * sample indices tile by tile (increasing within a tile), inv [n] int32 (may
 * be NULL) is its inverse, and tile_start [K+2] int64 (device) bounds the
 * groups: tile k is perm[tile_start[k] .. tile_start[k+1]); entries from
 * tile_start[K] to tile_start[K+1] = *n_dev (or n) hold samples whose tile
 * id is >= K (raising SNAKE_DEVERR_TILE_ID).  tile_id may be NULL when K == 1.
 * Optional gathers into the new order (each may be NULL): pos_out [n][3],
 * tile_out [n], ray_out [n].  1 <= K <= 16, n < 2^31.
 * Workspace: snake_tile_partition_workspace_bytes(K).
 */
size_t snake_tile_partition_workspace_bytes(int32_t K);
int snake_tile_partition(const uint8_t *tile_id, const float *pos, const int32_t *ray_id,
                         int64_t n, const int64_t *n_dev, int32_t K, int32_t *perm,
                         int32_t *inv, int64_t *tile_start, float *pos_out, uint8_t *tile_out,
                         int32_t *ray_out, void *workspace, size_t workspace_bytes,
                         snake_stream_t stream);

/*
 * Coarse occupancy grid and culling (the SAT-NGP procedure the paper follows
 * in training, Sec. 4.1).  Each of K tiles has a G^3 grid over its [0,1]^3
 * frame (G a power of two in [2, 1024]); a tile-frame position x lies in cell
 * c_a = min(floor(x_a G), G-1), flattened (c_x G + c_y) G + c_z, tile k's grid
 * at offset k G^3; occupancy is bit c % 32 of word c / 32.
 *
 * snake_occupancy_cells writes the centre ((i+.5)/G, (j+.5)/G, (k+.5)/G) of
 * every cell of the K grids (pos [K G^3][3]) and its tile id (tile_id may be
 * NULL), for evaluating the density there with the encoding and networks.
 * snake_occupancy_update folds the density sigma [n_cells] evaluated at the
 * cell centres into the grid: density [n_cells] float becomes
 * max(decay * density, sigma_scale * sigma) -- with sigma_scale the sample
 * step, the grid holds the optical thickness of one step -- and bits
 * [ceil(n_cells/32)] uint32 are set to density > thr, where thr = threshold,
 * or with SNAKE_OCC_MEAN_CAP in flags thr = min(threshold, mean of the new
 * density over the n_cells cells), so that while the whole field is thin the
 * denser half of it stays occupied.  The mean is summed in a fixed order in
 * compensated FP32 (value plus rounding error, about 2^-44 relative; the same
 * bits on every call).  decay in [0, 1], sigma_scale > 0.
 * Workspace: snake_occupancy_workspace_bytes(n_cells), 8-byte aligned.
 * snake_cull_samples keeps, ray by ray and in order, the packed samples
 * whose cell is occupied (a tile id >= K is dropped with
 * SNAKE_DEVERR_TILE_ID) and writes them packed again: packed_info_out [R][2],
 * t0/t1/pos/ray_id/tile_id outputs (tile_id_out may be NULL) for up to cap
 * samples, *n_out (device) = the kept total (SNAKE_DEVERR_CAPACITY past cap).
 * Culled intervals then add no optical depth to the quadrature.
 * Workspace: snake_cull_workspace_bytes(R).
 */
/*
 * snake_sample_refine gives each ray segment its sample density from the
 * grid (Sec. 4.1: the coarse grid's voxel density provides the sample
 * density of each ray segment).  After culling, a ray that kept c > 0 of its
 * samples spends its whole budget B -- its sample count before culling,
 * packed_info_all[r][1] -- on the kept intervals: interval i is split into
 * e(i+1) - e(i) equal sub-intervals, e(i) = floor((2 B i + c) / (2 c)) (so
 * each gets floor(B/c) or ceil(B/c)), with its sample at the sub-interval's
 * midpoint; a ray that kept nothing gets no samples.  Inputs: the rays and
 * boxes of the sampler call (FP64, device rays, host boxes [K][6]), the
 * sampler's packed_info_all [R][2] and the culled packed_info_kept [R][2],
 * t0_kept / t1_kept / tile_id_kept (tile_id_kept may be NULL when K == 1).
 * Outputs as for snake_sample_segmented (packed_info [R][2], t0, t1, pos
 * [n][3] in the tile frame, ray_id, tile_id (may be NULL), up to cap
 * samples, *n_out on the device; SNAKE_DEVERR_CAPACITY past cap).  Bounds and
 * positions use the sampler's FP32 rounding points, so with every interval
 * kept the result equals the sampler's.  Workspace:
 * snake_sample_workspace_bytes(R).
 */
int snake_sample_refine(const double *rays_o, const double *rays_d, int32_t R, const double *boxes, int32_t K,
                        const int32_t *packed_info_all, const int32_t *packed_info_kept, const float *t0_kept,
                        const float *t1_kept, const uint8_t *tile_id_kept, int32_t *packed_info, float *t0,
                        float *t1, float *pos, int32_t *ray_id, uint8_t *tile_id, int64_t cap, int64_t *n_out,
                        void *workspace, size_t workspace_bytes, snake_stream_t stream);
int snake_occupancy_cells(int32_t G, int32_t K, float *pos, uint8_t *tile_id, snake_stream_t stream);
#define SNAKE_OCC_MEAN_CAP 1u          /* threshold capped at the mean density */
size_t snake_occupancy_workspace_bytes(int64_t n_cells);
int snake_occupancy_update(const float *sigma, int64_t n_cells, float decay, float sigma_scale,
                           float threshold, uint32_t flags, float *density, uint32_t *bits,
                           void *workspace, size_t workspace_bytes, snake_stream_t stream);
size_t snake_cull_workspace_bytes(int32_t R);
int snake_cull_samples(int32_t G, const uint32_t *bits, int32_t K, int32_t R,
                       const int32_t *packed_info, const float *t0, const float *t1,
                       const float *pos, const int32_t *ray_id, const uint8_t *tile_id,
                       int32_t *packed_info_out, float *t0_out, float *t1_out, float *pos_out,
                       int32_t *ray_id_out, uint8_t *tile_id_out, int64_t cap, int64_t *n_out,
                       void *workspace, size_t workspace_bytes, snake_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Multiresolution hash encoding (Sec. 4.1; the NGP representation)          */
/* ------------------------------------------------------------------------ */

#define SNAKE_MAX_LEVELS 32
#define SNAKE_GRID_ALWAYS_HASH 1u      /* hash every level, even when dense fits */
#define SNAKE_GRID_TABLE_BF16 2u       /* forward: the table is a BF16 mirror */

typedef struct {
    int32_t n_levels;                  /* L, 1..32 */
    int32_t n_features;                /* F, 1, 2 or 4 */
    int32_t log2_table;                /* log2 T, 4..24 */
    int32_t feat_dtype;                /* snake_dtype of the feature array */
    uint32_t flags;                    /* SNAKE_GRID_* */
    int32_t resolution[SNAKE_MAX_LEVELS];  /* N_l >= 1 per level */
} snake_grid_desc;

/*
 * Level l of resolution N: p = fl32(x * N) per axis, cell c = min(floor p, N-1),
 * w = p - c; the 8 corners c + b (b in {0,1}^3, bit 0 = x) are stored at
 *   dense:  i + j (N+1) + k (N+1)^2                       if (N+1)^3 <= T
 *   hashed: (i*1 XOR j*2654435761 XOR k*805459861) mod 2^32 AND (T-1)
 * and feat[l][s][f] = sum_b w_b table[tile][l][idx_b][f] with
 * w_b = prod_a (b_a ? w_a : 1 - w_a).
 * table [K][L][T][F] float (1 <= K <= 256), or with SNAKE_GRID_TABLE_BF16 in
 * g->flags its bfloat16 mirror of the same layout (the FP32 table rounded by
 * snake_convert_bf16; the blend stays FP32), 16-byte aligned; pos [.][3]
 * float, tile_id (NULL = tile 0 for all; an id >= K gives zero features and
 * SNAKE_DEVERR_TILE_ID), feat [L][n][F] written (with F == 2 aligned to one
 * row, 4 bytes for bf16, 8 for float; else SNAKE_ERR_ALIGN).  idx_dbg (NULL or
 * [n][L][8] uint32) receives the corner slots.  The adjoint ignores the flag
 * (its dtable is always FP32).
 */
int snake_hashgrid_fwd(const snake_grid_desc *g, int32_t K, const void *table,
                       const float *pos, const uint8_t *tile_id, const int32_t *sample_idx,
                       int64_t n, const int64_t *n_dev, void *feat, uint32_t *idx_dbg,
                       snake_stream_t stream);

/* dst[i] = src[i] rounded to bfloat16 (nearest, ties to even; NaN stays NaN)
 * for n floats (n a multiple of 4; src 16-byte, dst 8-byte aligned): the
 * half-precision parameter copy that mixed-precision NGP training gathers
 * from, refreshed from the FP32 master table before each forward. */
int snake_convert_bf16(const float *src, int64_t n, void *dst, snake_stream_t stream);

/* Adjoint: dtable[tile][l][idx_b][f] += w_b * dfeat[l][s][f] for the K tiles
 * of dtable [K][L][T][F] float; dfeat [L][n][F] float (compact, indexed by j).
 * With a workspace the corner contributions are binned by table slot (count,
 * scan, scatter) and summed exactly in integers: each stored value -- one
 * corner's w_b * dfeat in FP32, or the FP32 sum of a run of consecutive
 * samples of a ray sharing the slot -- is rounded once to 20 significant bits
 * (relative error <= 2^-20) with an exponent at most 63 binades below the
 * level's largest |dfeat| (smaller values count as 0; values more than 37
 * binades below it are rounded to a multiple of 2^-56 times it), the values
 * are added exactly into 128-bit integer sums, and every table entry receives
 * its sum rounded once to FP32.  So each entry keeps its own relative
 * precision whatever the gradients' spread: |error| <= about 2^-20 times the
 * sum of |w_b * dfeat| over its contributions, plus the final FP32 rounding.
 * The result is deterministic (the same bits for any grid or scheduling).  A
 * level whose dfeat holds a non-finite value adds nothing and raises
 * SNAKE_DEVERR_NONFINITE.  The workspace size decides how many levels share a
 * pass (snake_hashgrid_bwd_workspace_bytes(g, K, n, levels_per_pass); one
 * level per pass is the minimum).  With workspace == NULL every contribution
 * is a direct FP32 atomic add, whose order, hence last bits, is not
 * deterministic.  A tile_id >= K contributes nothing and raises
 * SNAKE_DEVERR_TILE_ID.  Limits: 1 <= K <= 256, K*T <= 2^28; the binned form
 * needs 8 n < 2^31 and puts at most (2^31 - 1) / (8 n) levels in a pass. */
size_t snake_hashgrid_bwd_workspace_bytes(const snake_grid_desc *g, int32_t K, int64_t n,
                                          int32_t levels_per_pass);
int snake_hashgrid_bwd(const snake_grid_desc *g, int32_t K, const float *pos, const uint8_t *tile_id,
                       const int32_t *sample_idx, int64_t n, const int64_t *n_dev,
                       const float *dfeat, float *dtable, void *workspace, size_t workspace_bytes,
                       snake_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Density and colour networks (Sec. 4.1)                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_levels;        /* L of the encoding feeding the density net */
    int32_t n_features;      /* F of the encoding; L*F <= 32, the density input is
                                zero-padded to 32 */
    int32_t n_dir;           /* 3: view direction; 6: view + sun direction */
    int32_t colour_layers;   /* hidden layers of the colour net: 1 or 2 */
    int32_t colour_out;      /* 3: rgb = sigmoid(o); 4: rgb = sigmoid(o_0..2) sigmoid(o_3) */
    int32_t precision;       /* SNAKE_F32 or SNAKE_BF16 (MFMA with FP32 accumulation) */
    int32_t feat_dtype;      /* snake_dtype of the feature array */
    int32_t shared_colour;   /* 0: each NeRF tile has its own colour net; 1: one colour
                                net shared by the tiles of a call (Sec. 4.1: local
                                density networks, a global colour network) */
} snake_mlp_desc;

/* Fixed widths: density 32 -> 64 -> 16 (ReLU hidden, sigma = exp(o_0),
 * embedding o_1..o_15), colour [embedding, view, (sun)] -> 64 (-> 64) -> 3|4,
 * no biases.  Packed weight order: density L1 [64][32], density L2 [16][64],
 * colour L1 [64][15+n_dir], colour L2 [64][64] (if 2 layers), colour out
 * [colour_out][64]. */
int64_t snake_mlp_param_count(const snake_mlp_desc *m);

/* Floats of the weight (and weight-gradient) array for K tiles: K * P, or
 * with shared_colour the K density sets [K][Pd] (Pd = 64*32 + 16*64) followed
 * by one colour set [P - Pd].  -1 for a bad descriptor or K. */
int64_t snake_mlp_weight_count(const snake_mlp_desc *m, int32_t K);

/* Per-tile networks (the window step, Sec. 4.4): with K > 1, weights holds
 * snake_mlp_weight_count(m, K) floats (per-tile sets [K][P], or per-tile
 * density sets and one shared colour set) and tile_start [K+2] (device int64, as written by
 * snake_tile_partition) splits the call's entries j into groups; group k < K
 * uses weight set k, entries of group K are dropped (sigma = rgb = 0, dfeat =
 * 0), and dW has the layout of weights (a shared colour net's gradient sums
 * over all tiles).  K == 1 takes tile_start = NULL (one group [0, n)).
 * The groups are processed in 64-entry units that never mix two weight sets.
 * 1 <= K <= 16.
 *
 * Forward.  feat [L][n][F] (level-major; sample j's row is j), view/sun
 * [R][3] float per ray (sun may be NULL when n_dir == 3), ray_id per input
 * sample (read through sample_idx); a ray id outside [0, R) gives sigma = 0,
 * rgb = 0 and raises SNAKE_DEVERR_RAY_ID.  Writes sigma [n], rgb [n][3].  BF16
 * precision rounds inputs, weights and hidden activations to bf16 (RNE) and
 * accumulates in FP32.  With F == 2, feat is aligned to one row (2 elements);
 * a misaligned pointer returns SNAKE_ERR_ALIGN.
 * act: NULL, or [n][snake_mlp_act_width(m)] float (16-byte aligned) that
 * receives every sample's hidden and output activations for an adjoint
 * that does not recompute them (samples with a bad ray id are not written). */
int32_t snake_mlp_act_width(const snake_mlp_desc *m);
int snake_mlp_fwd(const snake_mlp_desc *m, int32_t K, const float *weights,
                  const int64_t *tile_start, const void *feat,
                  const float *view, const float *sun, const int32_t *ray_id, int32_t R,
                  const int32_t *sample_idx, int64_t n, const int64_t *n_dev,
                  float *sigma, float *rgb, float *act, snake_stream_t stream);

/* Adjoint.  act == NULL: activations are recomputed from feat; otherwise
 * they are read from act as stored by snake_mlp_fwd (read through
 * sample_idx like feat), with identical results.  feat, ray_id, dsigma
 * and drgb are read through sample_idx (feat level-major with level stride
 * feat_ld >= every index read); dfeat [L][n][F] float is written compact at
 * j (zero for a sample whose ray id is outside [0, R), which is flagged with
 * SNAKE_DEVERR_RAY_ID).  dW [P] += the sum over samples, reduced in a fixed
 * order (deterministic for a given n).  With F == 2, feat and dfeat are
 * aligned to one row.  Workspace: snake_mlp_bwd_workspace_bytes(m, K). */
size_t snake_mlp_bwd_workspace_bytes(const snake_mlp_desc *m, int32_t K);
int snake_mlp_bwd(const snake_mlp_desc *m, int32_t K, const float *weights,
                  const int64_t *tile_start, const void *feat,
                  int64_t feat_ld, const float *view, const float *sun, const int32_t *ray_id,
                  int32_t R, const int32_t *sample_idx, int64_t n, const int64_t *n_dev,
                  const float *dsigma, const float *drgb, const float *act, float *dW,
                  float *dfeat, void *workspace, size_t workspace_bytes, snake_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Volume rendering and colour-consistency loss (Sec. 2.2, 4.4, 4.5)         */
/* ------------------------------------------------------------------------ */

/*
 * Per ray: delta_i = t1_i - t0_i, T_i = exp(-sum_{j<i} sigma_j delta_j) (a
 * prefix product of exp(-sigma_j delta_j), taken as a prefix sum of optical
 * depth across the wavefront), alpha_i = 1 - exp(-sigma_i delta_i),
 * w_i = T_i alpha_i; rgb_out = sum w_i c_i, opacity = sum w_i,
 * depth = sum w_i (t0_i + t1_i)/2; background 0.  early_stop_T > 0 keeps only
 * the samples with T_i >= early_stop_T (a prefix); n_alive [R] (may be NULL)
 * receives the kept count.  With target [R][3] given, *loss (device float)
 * += loss_scale * sum_r sum_ch (rgb_out - target)^2, summed in a fixed order
 * (the same bits on every run).  opacity, depth, loss may be NULL.
 */
int snake_composite_fwd(const float *sigma, const float *rgb, const float *t0, const float *t1,
                        const int32_t *packed_info, int32_t R, const int32_t *sample_map,
                        float early_stop_T,
                        const float *target, float loss_scale,
                        float *rgb_out, float *opacity, float *depth, int32_t *n_alive,
                        float *loss, snake_stream_t stream);

/*
 * Adjoint of the loss above with g = 2 loss_scale (C - target):
 *   drgb_i = w_i g,  dsigma_i = delta_i sum_ch g_ch (T_{i+1} c_i,ch - (C_ch - A_i,ch)),
 * A_i = sum_{j<=i} w_j c_j, for i < n_alive[r] (all samples if n_alive is NULL);
 * the other samples of the ray get 0.  dsigma [N], drgb [N][3] written.
 *
 * sample_map (both calls; NULL = identity): packed sample p's sigma and rgb
 * are read at sample_map[p], and its dsigma and drgb written there, so the
 * per-sample arrays may be kept in another order (the tile-partitioned order
 * of the window step, sample_map = inv of snake_tile_partition) while t0, t1
 * and packed_info stay packed.
 */
int snake_composite_bwd(const float *sigma, const float *rgb, const float *t0, const float *t1,
                        const int32_t *packed_info, int32_t R, const int32_t *sample_map,
                        const int32_t *n_alive,
                        const float *target, float loss_scale,
                        float *dsigma, float *drgb, snake_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Adam (the I-NGP optimisation strategy, Sec. 4.6)                          */
/* ------------------------------------------------------------------------ */

#define SNAKE_ADAM_ZERO_GRAD 1u    /* write 0 to g after reading it */

/* g' = g + l2 p; m = b1 m + (1-b1) g'; v = b2 v + (1-b2) g'^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps), step >= 1.
 * p, g, m, v [n] float, 16-byte aligned.  The bias corrections are
 * 1 - b^step with b^step formed by binary powering in FP32 (the same bits
 * whether the step comes from the host or from step_dev).
 * step_dev: NULL, or a device int32 holding the step (then `step` is
 * ignored), so that a captured HIP graph replays with the current step;
 * snake_counter_add advances it inside the same graph. */
int snake_adam_step(float *p, float *g, float *m, float *v, int64_t n,
                    float lr, float b1, float b2, float eps, int32_t step,
                    const int32_t *step_dev, float l2, uint32_t flags, snake_stream_t stream);

/* Adam over K NeRF tiles in one launch (the window step, whose tiles keep
 * their own step counts, Sec. 4.4): p, g, m, v hold K consecutive blocks of
 * tile_n floats (4-byte aligned), and block k takes its step from step_dev[k]
 * (device int32; values below 1 count as 1).  Otherwise as snake_adam_step,
 * with the same bits as K separate calls.  1 <= K <= 64. */
int snake_adam_step_tiles(float *p, float *g, float *m, float *v, int64_t tile_n, int32_t K,
                          float lr, float b1, float b2, float eps, const int32_t *step_dev, float l2,
                          uint32_t flags, snake_stream_t stream);

/* counter[i] += delta for i < n on the stream (device int32 [n]; per-tile
 * Adam step counters). */
int snake_counter_add(int32_t *counter, int32_t n, int32_t delta, snake_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SNAKE_H */
