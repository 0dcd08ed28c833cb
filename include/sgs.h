/*
 * sgs.h -- C ABI of the MI355X (gfx950) rasterizer for 3D skew Gaussians.
 *
 * The library renders scenes of 3D skew Gaussians (paper: "3D Skew Gaussian
 * Splatting", Sec. "3D Skew Gaussian Kernel" S(x) = 2 G(x) Phi(beta^T(x-mu)))
 * with a tile-based pipeline, forward and backward:
 *
 *   sgs_preprocess  per (view, Gaussian): covariance, EWA projection, 2D skew,
 *                   SH colour, skew-aware screen extent, tile count, and the
 *                   prefix sum of tile counts (instance count on the device).
 *   sgs_bin_sort    one (tile, depth) key per covered tile, stable LSD radix
 *                   sort, per-tile ranges of the sorted list.
 *   sgs_render_fwd  per-tile front-to-back compositing (Alg. 1).
 *   sgs_render_bwd  reverse-order blend backward (Alg. 2) and the chain rule
 *                   back to the 3D parameters (Sec. "3D Skew Gaussian
 *                   Rasterization and Splatting", gradient of the loss w.r.t.
 *                   beta; appendix "Backward Pass").
 *
 * Conventions (all calls):
 *  - Every pointer named *_dev or documented as "device" is device memory on
 *    the current HIP device; everything else is host memory.  Device arrays are
 *    float32 structure-of-arrays unless stated: a field "[k][n]" stores
 *    component j of element i at index j*n + i.
 *  - The caller allocates and owns all memory, including scratch; the library
 *    allocates nothing, keeps no global state and may be called concurrently
 *    on distinct streams with distinct buffers.  The one exception is
 *    sgs_bin_sort_noalloc, which uses a fixed scratch array held by the
 *    library on each device (see there).
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue
 *    work and return; no call synchronises.  Kernel launch errors are reported
 *    as SGS_EHIP by the call that launched them.
 *  - Gradient outputs are accumulated (+=); the caller zeroes them.
 *  - Degenerate Gaussians (behind the near plane, singular 2D covariance,
 *    non-finite values, too faint to reach alpha_min anywhere) are culled
 *    silently: zero tiles, no output, zero gradient.  Never an error.
 */
#ifndef SGS_H
#define SGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGS_OK = 0,
  SGS_EINVAL = 1,      /* null required pointer, bad size or option        */
  SGS_ECAPACITY = 2,   /* caller buffer smaller than the size helper asks  */
  SGS_EHIP = 3,        /* HIP runtime / launch error                       */
  SGS_EUNSUPPORTED = 4 /* valid but not implemented (e.g. tile shape)      */
} sgs_status;

/* Gaussian parameters, device pointers (Sec. "Preliminary of 3D Gaussian
 * Splatting": mean, scale, rotation quaternion, opacity, SH colour; Sec. "3D
 * Skew Gaussian Kernel": skew vector beta in R^3; Sec. "3D Skew Gaussian
 * Rasterization and Splatting": enhanced opacity with two base opacities and
 * a direction). */
typedef struct {
  int64_t n;               /* number of Gaussians N >= 0                    */
  int32_t sh_degree;       /* 0..3, K = (sh_degree+1)^2 coefficients        */
  int32_t _pad;
  const float* mean;       /* [3][N] world position                         */
  const float* log_scale;  /* [3][N] log of the per-axis scale              */
  const float* quat;       /* [4][N] rotation (w,x,y,z), any non-zero norm  */
  const float* skew;       /* [3][N] beta, or NULL: symmetric 3DGS path     */
  const float* opa_logit;  /* [N]    logit of base opacity alpha_1          */
  const float* opa2_logit; /* [N]    logit of alpha_2, or NULL (alpha_2 = alpha_1,
                                     enhanced opacity off)                  */
  const float* opa_dir;    /* [3][N] direction d of the enhanced opacity, or
                                     NULL (d = 0); used only with opa2_logit */
  const float* sh;         /* [K][3][N] SH coefficients                     */
} sgs_params;

/* Accumulated (+=) gradients, device pointers, same shapes as sgs_params.
 * Any pointer may be NULL (that output is skipped).
 *
 * The last three fields are the per-Gaussian statistics that drive
 * densification (Sec. "Depth-Aware Densification Strategy", Eq. depth_grad),
 * gathered by the backward of each call over its n views v, where L_v is
 * view v's part of the loss and a view "sees" a Gaussian when its extent
 * covers at least one tile:
 *   densify_uv[i]    += sum over seeing views of the screen-space gradient
 *                       norm || (dL_v/dmu2d_x * W_v/2, dL_v/dmu2d_y * H_v/2) ||
 *                       (NDC units, the 2D statistic g_uv)
 *   densify_z[i]      = max(densify_z[i], max over seeing views of
 *                       | r_v . dL_v/dmean |), r_v the third row of view v's
 *                       w2c: the gradient w.r.t. the depth of the centre (g_z)
 *   densify_count[i] += number of seeing views
 * The caller zeroes them once per densification interval. */
typedef struct {
  float* mean;
  float* log_scale;
  float* quat;
  float* skew;
  float* opa_logit;
  float* opa2_logit;
  float* opa_dir;
  float* sh;
  float* densify_uv;        /* [N] or NULL */
  float* densify_z;         /* [N] or NULL */
  uint32_t* densify_count;  /* [N] or NULL */
} sgs_params_grad;

/* One pinhole view in the OpenCV convention (+x right, +y down, +z forward;
 * Sec. "Camera Trajectories and Format Standardization").  Build it from a
 * frontend (OpenGL/Blender) pose with sgs_camera_from_gl; lay a batch out
 * with sgs_camera_layout.  The same array is passed to the library twice:
 * in host memory (sizes, grids) and as an identical copy in device memory
 * (read by the kernels). */
typedef struct {
  int32_t width, height;   /* pixels, > 0                                   */
  float fx, fy, cx, cy;    /* intrinsics K                                  */
  float w2c[12];           /* row-major 3x4 world-to-camera [R|t]           */
  float campos[3];         /* camera centre in world coordinates            */
  float near_z;            /* Gaussians with camera z <= near_z are culled  */
  float bg[3];             /* background colour                             */
  int32_t tiles_x, tiles_y;/* set by sgs_camera_layout                      */
  int32_t tile_base;       /* first global tile id of this view             */
  int64_t pix_base;        /* first pixel of this view in the output planes */
} sgs_camera;

/* Instance capacity from which sort_mode -1 runs mode 2 (393,216: on
 * clustered scenes at 1280x720 the two modes cross between 0.32M and 0.37M
 * instances of capacity; mode 2 ran 0.2-1.2% faster from 0.37M to 0.96M and
 * far faster at 65M, mode 1 0.8-1.8% faster below 0.32M). */
#define SGS_AUTO_ROWBIN_CAPACITY ((int64_t)3 << 17)

/* Pipeline options; sgs_default_options fills the values in brackets. */
typedef struct {
  int32_t tile_w, tile_h;  /* [16, 16]; also 16x8 and 8x8                  */
  float filter_s;          /* [0.3] low-pass filter added to Sigma' (px^2)  */
  int32_t compensate;      /* [1] opacity compensation sqrt(det S'/det(S'+sI)) */
  float guard;             /* [1.3] Jacobian clamp of x/z, y/z in tan(fov/2) */
  float alpha_min;         /* [1/255] pairs below are skipped               */
  float alpha_max;         /* [0.99] alpha clamp                            */
  float t_min;             /* [1e-4] a pixel stops before T drops below     */
  int32_t sort_mode;       /* [-1] 0: 64-bit (tile<<32 | depth) keys, one LSD
                              sort; 1: stable depth presort of the records,
                              duplicate in depth order, LSD sort of 32-bit
                              tile keys; 2: depth presort, one item per
                              non-empty tile row of each record, stable sort
                              of the items by tile row, then each row's
                              items placed into its tiles (needs
                              sgs_geom.rows, at most 64 views, 256 tiles per
                              row and 65536 tile rows per call; otherwise
                              mode 1 runs); -1: mode 2 from an instance
                              capacity of SGS_AUTO_ROWBIN_CAPACITY up, else
                              mode 1 (measured faster at small sizes).  All
                              give the identical order.                     */
  int32_t blend_batch;     /* [0] records staged in LDS per batch: 64, 128, 256; 0: 128 in the
                              forward blend, 256 in the backward */
  int32_t split_tiles;     /* [-1] with 16x16 tiles and a tile order (and no
                              work counter): both blends run the first
                              split_tiles tiles of the order (the longest
                              lists) as four 8x8 quarters, four lanes per
                              pixel evaluating four records at once; same
                              images (gradients up to the order of float
                              sums), more parallelism per tile.  -1:
                              total_tiles / 128; 0: off.                    */
  int32_t depth_digit_bits;/* [0] radix digits of the depth presort (sort
                              mode 1): 8 (4 passes over the 32-bit keys),
                              10 (3 passes over keys shifted to 30 bits; needs
                              every near_z > 0 and at most 16.7M records,
                              else 8 is used), 0: 8 (the fewer, wider
                              passes measured slower on gfx950: each pass's
                              LDS ranking grows with the digit).  Same order
                              either way.                                   */
  int32_t blend_lists;     /* [0] record lists of the forward blend's tiles
                              (Alg. 1 walks a tile's records front to back;
                              a list holds the ones whose extent reaches a
                              pixel block): 1, one per wave's 8x8 block; 4,
                              one per 4x4 quarter of it (fewer steps where
                              records are small, each step dearer); 0: 4
                              when the instance capacity is at most 8 per
                              record, else 1.  Same images either way.      */
} sgs_options;

/* Projected per-record data written by sgs_preprocess, record m = v*N + i for
 * view v and Gaussian i (M = n_views * N records).  Device pointers; sizes
 * from sgs_geom_rec_floats.  `rec` holds one 64-byte entry of four float4
 * slots per record (a record is gathered whole by index, so one entry is
 * one cache line):
 *   slot 0: (mu_x, mu_y, a, b)   2D mean in pixels, conic (Sigma'+sI)^-1 = [[a,b],[b,c]]
 *   slot 1: (c, beta_x, beta_y, d)  2D skew; d = rho*alpha_1 (rho with enhanced opacity)
 *   slot 2: (r, g, b, log_thr)   colour; log_thr: below this exponent a pair is skipped
 *   slot 3: (alpha_1, alpha_2, w_x, w_y)  with enhanced opacity; otherwise the
 *           two words of the record's tile rect (as in `rect`) in .x and .y,
 *           so that binning gathers one 64-byte line per record
 * `enhanced` says which: it must equal (p->opa2_logit != NULL) of the
 * parameters passed to sgs_preprocess (EINVAL otherwise).
 */
typedef struct {
  float* rec;              /* [M][4][4]                                     */
  float* depth;            /* [M] camera-space z (the sort key); all-ones
                              bits (a NaN) for records without tiles       */
  uint32_t* rect;          /* [M][2] tile rect: (x0 | y0<<16, x1 | y1<<16), half-open */
  uint32_t* tiles;         /* [M] number of tiles covered (0 = culled)      */
  uint32_t* block_off;     /* [sgs_geom_block_entries(N, V)] exclusive prefix of the
                              tile counts per block of 256 records of one view
                              (view-major); the last entry is the total      */
  uint32_t* rows;          /* [M] number of tile rows of the rect with at
                              least one covered tile (0 = culled); written
                              when non-NULL, needed by sort_mode 2          */
  int32_t enhanced;        /* 1: records carry enhanced opacity (slot 3)   */
  int32_t _pad;
} sgs_geom;

/* Optional tile scheduling for the blend kernels (device pointers).
 *  tile_order    [total_tiles] u32: written by sgs_bin_sort when non-NULL, a
 *                permutation of the tile ids by decreasing list length on a
 *                quarter-octave scale (longest first, so the slowest tiles
 *                start first; the order inside a length bucket is
 *                unspecified); read by the blends, which then take tiles in
 *                this order.  It changes scheduling only, never results.
 *  work_counter  [1] u32: when non-NULL the blends run persistent workgroups
 *                (as many as fit on the device) that take the next tile from
 *                this counter until all tiles are done; the call resets it on
 *                the stream before the kernel.  NULL: one workgroup per tile. */
typedef struct {
  uint32_t* tile_order;
  uint32_t* work_counter;
} sgs_schedule;

/* Accumulated (+=) gradient of the loss w.r.t. the projected records, same
 * [R][M][4] planes (R = 3, or 4 with enhanced opacity): plane k holds the
 * gradients of record slot k of sgs_geom.rec (plane 2 .w unused).  Device
 * pointer, sgs_geom_rec_floats(M, enhanced) floats. */
typedef struct {
  float* rec;
} sgs_geom_grad;

/* ---------------------------------------------------------------- helpers */
void sgs_default_options(sgs_options* opt);

/* sizeof of the ABI structs, for bindings to check their mirrors:
 * 0 sgs_params, 1 sgs_params_grad, 2 sgs_camera, 3 sgs_options, 4 sgs_geom,
 * 5 sgs_geom_grad, 6 sgs_schedule, 7 sgs_adam_group, 8 sgs_densify_options,
 * 9 sgs_densify_out; 0 for any other value. */
size_t sgs_struct_size(int32_t which);
const char* sgs_status_string(sgs_status s);

/* CoordEngine and intrinsic mapping (Alg. 3; Sec. "Decoupled Interactive
 * Visual Analytics Engine"): M_cv = M_gl T_align, T_align = diag(1,-1,-1,1);
 * w2c = M_cv^-1; K = [[W/(2tan(fovx/2)),0,W/2],[0,H/(2tan(fovy/2)),H/2]].
 * c2w_gl: row-major 4x4 OpenGL camera-to-world (host).  fovy_rad <= 0 means
 * square pixels (fy = fx).  Fills every field except the layout fields.
 * EINVAL for non-finite input, W or H <= 0, fov outside (0, pi). */
sgs_status sgs_camera_from_gl(const double c2w_gl[16], int32_t width, int32_t height,
                              double fovx_rad, double fovy_rad, float near_z,
                              const float bg[3], sgs_camera* out);

/* Lays n_views cameras (host array) out in one global tile and pixel space:
 * sets tiles_x, tiles_y, tile_base, pix_base; returns the totals. */
sgs_status sgs_camera_layout(sgs_camera* cams, int32_t n_views, const sgs_options* opt,
                             int64_t* total_tiles, int64_t* total_pixels);

/* Float counts of the buffers of sgs_geom / sgs_geom_grad for M records. */
int64_t sgs_geom_rec_floats(int64_t m, int32_t enhanced);
int64_t sgs_geom_block_entries(int64_t n, int32_t n_views);

/* Scratch bytes sgs_bin_sort needs for M records, an instance capacity and a
 * number of tiles (same options). */
size_t sgs_bin_sort_scratch_bytes(int64_t m, int64_t inst_capacity, int64_t total_tiles,
                                  const sgs_options* opt);

/* The sort mode (0, 1 or 2) sgs_bin_sort runs for these options, capacity
 * and cameras (host array), given whether sgs_geom.rows is set; -1 for
 * arguments sgs_bin_sort rejects.  For reports and tests: the results are
 * the same in every mode. */
int32_t sgs_bin_sort_mode(const sgs_options* opt, int64_t inst_capacity, const sgs_camera* cams_host,
                          int32_t n_views, int32_t have_rows);

/* ------------------------------------------------------------------ calls */

/* Projects every Gaussian into every view (see sgs_geom) and computes
 * block_off (scan of the tile counts), so that *block_off[last] is the
 * number of instances.  Per (view, Gaussian), in the paper's terms:
 *  - Sigma = R S S^T R^T from the normalised quaternion and exp(log_scale),
 *    opacity sigmoid(logit), colour from the SH coefficients in the view
 *    direction (Sec. "Preliminary of 3D Gaussian Splatting");
 *  - world-to-camera with the view's w2c (M_cv of Alg. 3), cull at
 *    z <= near_z, depth = camera z;
 *  - Sigma' = J W Sigma W^T J^T (the affine EWA approximation of the same
 *    section), conic (Sigma' + s I)^-1 and opacity compensation
 *    sqrt(det Sigma' / det(Sigma' + s I)) (appendix "Forward Pass", Alg. 1);
 *  - the 2D skew (beta_x, beta_y) of Alg. 1 from the 3D skew vector of
 *    Sec. "3D Skew Gaussian Kernel", as the skew-normal marginal under the
 *    same affine map and filter;
 *  - the extent where alpha can reach alpha_min (the Gaussian's ellipse,
 *    cut by the half-plane where 1 + erf(z) is large enough) as a tile rect
 *    and an exact per-row tile count.
 * cams_host / cams_dev: the same n_views laid-out cameras.  Outputs in g
 * (caller-allocated, sizes from sgs_geom_rec_floats and
 * sgs_geom_block_entries); every entry is overwritten.  The instance count
 * in block_off saturates at 0xffffffff (more than one sort launch can
 * take).  EINVAL: null pointers, n < 0, sh_degree > 3, bad options or
 * cameras; EUNSUPPORTED: n * n_views >= 2^32 records. */
sgs_status sgs_preprocess(const sgs_params* p, const sgs_camera* cams_host,
                          const sgs_camera* cams_dev, int32_t n_views,
                          const sgs_options* opt, const sgs_geom* g, void* stream);

/* The tile pipeline's duplication and sort (Sec. "Preliminary of 3D
 * Gaussian Splatting": a tile-based pipeline blends each pixel's Gaussians
 * in near-to-far order; Alg. 1 walks each tile's list front to back).  Writes,
 * for each record with tiles > 0 and each tile its extent reaches
 * (row-major inside its rect: per tile row, the columns whose pixel centres
 * the evaluation ellipse reaches, cut by the skew half-plane), one instance,
 * sorts them stably by (global tile, depth) (ties keep record order) and
 * extracts tile_ranges[t] = [start, end).  One call sorts at most
 * 2^32 - 2 instances (32-bit positions and counts).
 *  keys          [inst_capacity] u64 (tile<<32 | float bits of depth), sorted;
 *                may be NULL (then not written) in sort_mode 1.
 *  vals          [inst_capacity] u32 record index m, sorted.
 *  tile_ranges   [total_tiles][2] u32.
 *  n_inst_dev    [1] u32 device: receives the instance count.  Instances past
 *                inst_capacity are dropped; the caller compares the count with
 *                the capacity after the fact (graph-friendly, no host sync).
 *                0xffffffff marks an internal failure (a sort look-back that
 *                did not complete in bounded time): the outputs are invalid.
 *  sched         optional (NULL): if sched->tile_order is set, it is written.
 *  scratch       device, >= sgs_bin_sort_scratch_bytes(...).
 * EINVAL / ECAPACITY for bad sizes. */
sgs_status sgs_bin_sort(const sgs_geom* g, int64_t m, const sgs_camera* cams_host,
                        const sgs_camera* cams_dev, int32_t n_views,
                        const sgs_options* opt, int64_t inst_capacity,
                        uint64_t* keys, uint32_t* vals, uint32_t* tile_ranges,
                        uint32_t* n_inst_dev, const sgs_schedule* sched, void* scratch,
                        size_t scratch_bytes, void* stream);

/* sgs_bin_sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, checks, results and errors as sgs_bin_sort, minus the
 * scratch pair: the scratch is a fixed array of SGS_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per device, part of the library's code object, allocated when the
 * library is loaded on that device and held until the process ends.  The
 * call itself allocates nothing (no hipMalloc, no allocating library
 * routine); its first call on a device looks up the array's address there.
 *  - ECAPACITY when sgs_bin_sort_scratch_bytes(m, inst_capacity, tiles, opt)
 *    exceeds SGS_NOALLOC_SCRATCH_BYTES (at 3600 tiles about 1.19M records
 *    with twice as many instances of capacity fit, 1.27M in sort mode 1; the
 *    300k-Gaussian 1280x720 frame needs 20.3 MiB, 14.5 MiB in mode 1),
 *    checked before any work is enqueued.
 *  - Every call on one device shares that device's array and clears what it
 *    needs at its start (on the stream, with a fill kernel).  Calls that
 *    overlap in time on one device race on it: serialise them (one stream, or
 *    events between streams). */
#define SGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sgs_status sgs_bin_sort_noalloc(const sgs_geom* g, int64_t m, const sgs_camera* cams_host,
                                const sgs_camera* cams_dev, int32_t n_views,
                                const sgs_options* opt, int64_t inst_capacity, uint64_t* keys,
                                uint32_t* vals, uint32_t* tile_ranges, uint32_t* n_inst_dev,
                                const sgs_schedule* sched, void* stream);

/* Alg. 1 per pixel: alpha = min(alpha_max, d G'(x) (1 + erf(beta.delta/sqrt2)))
 * (times the enhanced-opacity factor), pairs below alpha_min skipped, stop
 * before T falls below t_min; C += c alpha T.  vals / tile_ranges as written
 * by sgs_bin_sort with the same inst_capacity (ranges are clamped to it).  Outputs (device, per view at
 * its pix_base): out_rgb planes [3][P] (colour + T_final*bg), out_T [P]
 * (final transmittance), out_last [P] (number of range entries up to and
 * including the last contributor, 0 if none), and two optional work
 * counters (NULL to skip; with both NULL the blend runs without counting):
 * out_count [P] pairs composited into the pixel, out_eval [P] pairs
 * evaluated for it (alpha computed: past the exponent test of the skip
 * rule, before the comparison with alpha_min). */
sgs_status sgs_render_fwd(const sgs_geom* g, int64_t m, const uint32_t* vals,
                          int64_t inst_capacity, const uint32_t* tile_ranges,
                          const sgs_schedule* sched, const sgs_camera* cams_host,
                          const sgs_camera* cams_dev, int32_t n_views, int32_t enhanced,
                          const sgs_options* opt, float* out_rgb, float* out_T,
                          uint32_t* out_last, uint32_t* out_count, uint32_t* out_eval,
                          int64_t total_pixels, void* stream);

/* Alg. 2 and the chain rule.  Re-walks each pixel's list from its last
 * contributor to the front, rebuilding T from out_T (nothing per pair is
 * stored), accumulates the 2D record gradients g2d (reduced per tile in
 * registers/LDS before one atomic add per record and tile), then chains them
 * to the 3D parameters (grad, +=).  dL_drgb has the layout of out_rgb.
 * g2d must be zeroed by the caller before the call. */
sgs_status sgs_render_bwd(const sgs_params* p, const sgs_geom* g, int64_t m,
                          const uint32_t* vals, int64_t inst_capacity,
                          const uint32_t* tile_ranges, const sgs_schedule* sched,
                          const sgs_camera* cams_host, const sgs_camera* cams_dev,
                          int32_t n_views, const sgs_options* opt, const float* out_T,
                          const uint32_t* out_last, const float* dL_drgb,
                          int64_t total_pixels, const sgs_geom_grad* g2d,
                          const sgs_params_grad* grad, void* stream);

/* ------------------------------------------------------- densification */

/* Options of sgs_densify; sgs_default_densify_options fills the values in
 * brackets. */
typedef struct {
  float tau_uv;            /* [0.001] threshold of the mean screen-space
                              gradient norm (the appendix's tau_uv)        */
  float tau_z;             /* [0.001] threshold of the depth gradient g_z
                              (not given by the paper: a reading)          */
  float dense_scale;       /* [0.01] selected Gaussians whose largest scale
                              exceeds it are split, the others cloned
                              (3DGS: 0.01 x the scene extent)              */
  float split_shrink;      /* [1.6] child scale along the split axis is the
                              parent's divided by this (3DGS's factor)     */
} sgs_densify_options;

/* Output Gaussian set of sgs_densify: SoA arrays of `capacity` entries
 * (component j of entry o at j * capacity + o), same fields as sgs_params
 * (skew / opa2_logit / opa_dir may be NULL when the input has none), plus
 * the input index each output came from (NULL: not written). */
typedef struct {
  int64_t capacity;
  float* mean;
  float* log_scale;
  float* quat;
  float* skew;
  float* opa_logit;
  float* opa2_logit;
  float* opa_dir;
  float* sh;
  uint32_t* parent;
} sgs_densify_out;

void sgs_default_densify_options(sgs_densify_options* o);

/* Scratch words (u32) of sgs_densify for n Gaussians. */
int64_t sgs_densify_scratch_words(int64_t n);

/* The densification step of the training loop (Sec. "Depth-Aware
 * Densification Strategy", Eq. depth_grad; the appendix's tau_uv), from the
 * statistics the backward accumulates in sgs_params_grad.densify_*.
 * Decision per Gaussian i, in float32 (decision[i]: 0 keep, 1 clone,
 * 2 split):
 *   selected = uv_sum[i] / view_count[i] >= tau_uv (0 when the count is 0)
 *              or z_max[i] >= tau_z;
 *   split when selected and its largest log-scale > log(dense_scale),
 *   clone when selected otherwise.
 * The new set, in input order: a kept Gaussian once, a cloned one twice,
 * a split one as two children.  The split is along the largest scale axis
 * e and adjusts the children to the skew (the paper's split figure): each
 * child has scale s_max / split_shrink along e and the parent's other
 * scales, rotation, skew, opacities and SH; with delta = Sigma beta /
 * sqrt(1 + beta^T Sigma beta) of the parent and delta_c of a child, they sit
 * at mu + sqrt(2/pi) (delta - delta_c) +- a e with
 * a^2 = max(0, v - v_c), v = s_max^2 - (2/pi) (e.delta)^2 and
 * v_c = s_c^2 - (2/pi) (e.delta_c)^2: the pair's mean is the parent's and
 * its variance along e the parent's.
 *  uv_sum, view_count, z_max  [N] device (uv_sum and view_count together, or
 *                both NULL; z_max may be NULL: that criterion is off).
 *  decision      [N] u8 device, written.
 *  out           outputs past out->capacity are dropped; capacity 0 computes
 *                the decisions and the count only.
 *  n_out_dev     [1] u32 device: number of outputs (N + clones + splits).
 *  scratch       device, sgs_densify_scratch_words(N) u32 words.
 * EINVAL: null required pointers, n < 0, bad options. */
sgs_status sgs_densify(const sgs_params* p, const float* uv_sum, const uint32_t* view_count,
                       const float* z_max, const sgs_densify_options* opt, uint8_t* decision,
                       const sgs_densify_out* out, uint32_t* n_out_dev, uint32_t* scratch,
                       void* stream);

/* ---------------------------------------------------------- optimiser */

/* One parameter array of an Adam step (device pointers, n floats each). */
typedef struct {
  float* param;            /* updated in place                              */
  const float* grad;       /* gradient of the loss                          */
  float* m1;               /* first-moment estimate (zeroed before step 1)  */
  float* m2;               /* second-moment estimate (zeroed before step 1) */
  int64_t n;
  float lr;                /* learning rate of this array                   */
  int32_t _pad;
} sgs_adam_group;

#define SGS_ADAM_MAX_GROUPS 16

/* One Adam step (Kingma & Ba, ICLR 2015) over n_groups <= 16 arrays: the
 * optimiser of the training loop, which fits the Gaussian attributes by
 * gradient descent on the photometric loss (Sec. "Preliminary of 3D
 * Gaussian Splatting"; the appendix sets the skew's learning rate).  Per
 * element, with t the step count after this call:
 *   m1 = b1 m1 + (1 - b1) g;  m2 = b2 m2 + (1 - b2) g^2;
 *   param -= lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps).
 * state: 4 floats of device memory, zeroed before the first step; the call
 * advances state[0] = t and keeps the bias corrections in state[1..2] on the
 * device, so a captured graph of a training step replays correctly.
 * groups is a host array.  EINVAL: bad counts, null pointers, n < 0. */
sgs_status sgs_adam_step(const sgs_adam_group* groups, int32_t n_groups, float* state,
                         float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SGS_H */
