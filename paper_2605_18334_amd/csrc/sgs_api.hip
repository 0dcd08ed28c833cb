// extern "C" entry points of libsgs: argument checks and dispatch to the
// kernel launchers.  No allocation and no synchronisation.  The only global
// state is the fixed scratch array of sgs_bin_sort_noalloc and its per-device
// addresses (below).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "sgs_dev.h"

namespace sgs {
sgs_status launch_preprocess(const sgs_params*, const sgs_camera*, int32_t, const sgs_options*,
                             const sgs_geom*, hipStream_t);
sgs_status launch_preprocess_bwd(const sgs_params*, const sgs_camera*, int32_t,
                                 const sgs_options*, const sgs_geom*, const float*,
                                 const sgs_params_grad*, hipStream_t);
size_t bin_sort_scratch_bytes(int64_t m, int64_t cap, int64_t total_tiles, int mode);
sgs_status launch_bin_sort(const sgs_geom*, int64_t m, int64_t n, const sgs_camera*, int32_t,
                           int64_t total_tiles, const sgs_options*, int64_t cap, uint64_t*,
                           uint32_t*, uint32_t*, uint32_t*, uint32_t* tile_order, void*,
                           float near_min, int32_t rb_rows, int32_t rb_tx, hipStream_t);
sgs_status launch_blend_fwd(const sgs_geom*, int64_t, const uint32_t*, int64_t, const uint32_t*,
                            const sgs_schedule*, const sgs_camera*, int32_t, int64_t, int,
                            const sgs_options*, float*, float*, uint32_t*, uint32_t*, uint32_t*,
                            int64_t, hipStream_t);
sgs_status launch_blend_bwd(const sgs_geom*, int64_t, const uint32_t*, int64_t, const uint32_t*,
                            const sgs_schedule*, const sgs_camera*, int32_t, int64_t, int,
                            const sgs_options*, const float*, const uint32_t*, const float*,
                            int64_t, float*, hipStream_t);
sgs_status launch_adam(const sgs_adam_group*, int32_t, float*, float, float, float, hipStream_t);
sgs_status launch_densify(const sgs_params*, const float*, const uint32_t*, const float*,
                          const sgs_densify_options*, uint8_t*, uint32_t*, const sgs_densify_out*,
                          uint32_t*, hipStream_t);
}  // namespace sgs

namespace {

bool options_ok(const sgs_options* o) {
  if (!o) return false;
  const bool tile = (o->tile_w == 16 && o->tile_h == 16) || (o->tile_w == 16 && o->tile_h == 8) ||
                    (o->tile_w == 8 && o->tile_h == 8);
  const bool batch = o->blend_batch == 0 || o->blend_batch == 64 || o->blend_batch == 128 ||
                     o->blend_batch == 256;
  return tile && batch && isfinite(o->filter_s) && o->filter_s >= 0.0f && isfinite(o->guard) &&
         o->guard > 0.0f && o->alpha_min > 0.0f && o->alpha_min < o->alpha_max &&
         o->alpha_max < 1.0f && o->t_min > 0.0f && o->t_min < 1.0f &&
         (o->sort_mode >= -1 && o->sort_mode <= 2) && o->split_tiles >= -1 &&
         (o->depth_digit_bits == 0 || o->depth_digit_bits == 8 || o->depth_digit_bits == 10) &&
         (o->blend_lists == 0 || o->blend_lists == 1 || o->blend_lists == 4);
}

bool params_ok(const sgs_params* p) {
  return p && p->n >= 0 && p->n < ((int64_t)1 << 31) && p->sh_degree >= 0 && p->sh_degree <= 3 &&
         (p->n == 0 || (p->mean && p->log_scale && p->quat && p->opa_logit && p->sh));
}

bool cams_ok(const sgs_camera* c, int32_t n_views) {
  if (!c || n_views <= 0) return false;
  int64_t tb = 0, pb = 0;
  for (int v = 0; v < n_views; ++v) {
    const sgs_camera& k = c[v];
    if (k.width <= 0 || k.height <= 0 || k.width > 65535 * 8 || k.height > 65535 * 8) return false;
    if (!(isfinite(k.fx) && isfinite(k.fy) && isfinite(k.cx) && isfinite(k.cy) && k.fx > 0 && k.fy > 0))
      return false;
    for (float x : k.w2c)
      if (!isfinite(x)) return false;
    if (k.tile_base != tb || k.pix_base != pb || k.tiles_x <= 0 || k.tiles_y <= 0) return false;
    tb += (int64_t)k.tiles_x * k.tiles_y;
    pb += (int64_t)k.width * k.height;
  }
  return tb < ((int64_t)1 << 31);
}

int64_t tiles_total(const sgs_camera* c, int32_t n_views) {
  const sgs_camera& k = c[n_views - 1];
  return (int64_t)k.tile_base + (int64_t)k.tiles_x * k.tiles_y;
}

int64_t pixels_total(const sgs_camera* c, int32_t n_views) {
  const sgs_camera& k = c[n_views - 1];
  return k.pix_base + (int64_t)k.width * k.height;
}

// Scratch of sgs_bin_sort_noalloc: one array per device, allocated when the
// code object is loaded and held until the process ends.  In host code the
// name below only stands for the symbol; its device address comes from
// hipGetSymbolAddress, once per device (with that device current), and is
// the only handle host code ever passes on.
static __device__ __align__(256) unsigned char scratch[SGS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES];   // device address of `scratch` on each device

sgs_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SGS_EHIP;
  if (dev < 0 || dev >= MAX_DEVICES) return SGS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SGS_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SGS_OK;
}

}  // namespace

extern "C" {

void sgs_default_options(sgs_options* o) {
  if (!o) return;
  o->tile_w = 16;
  o->tile_h = 16;
  o->filter_s = 0.3f;
  o->compensate = 1;
  o->guard = 1.3f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->sort_mode = -1;
  o->blend_batch = 0;
  o->split_tiles = -1;
  o->depth_digit_bits = 0;
  o->blend_lists = 0;
}

size_t sgs_struct_size(int32_t which) {
  switch (which) {
    case 0: return sizeof(sgs_params);
    case 1: return sizeof(sgs_params_grad);
    case 2: return sizeof(sgs_camera);
    case 3: return sizeof(sgs_options);
    case 4: return sizeof(sgs_geom);
    case 5: return sizeof(sgs_geom_grad);
    case 6: return sizeof(sgs_schedule);
    case 7: return sizeof(sgs_adam_group);
    case 8: return sizeof(sgs_densify_options);
    case 9: return sizeof(sgs_densify_out);
  }
  return 0;
}

const char* sgs_status_string(sgs_status s) {
  switch (s) {
    case SGS_OK: return "ok";
    case SGS_EINVAL: return "invalid argument";
    case SGS_ECAPACITY: return "buffer too small";
    case SGS_EHIP: return "HIP error";
    case SGS_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

sgs_status sgs_camera_from_gl(const double c2w_gl[16], int32_t width, int32_t height,
                              double fovx_rad, double fovy_rad, float near_z, const float bg[3],
                              sgs_camera* out) {
  if (!c2w_gl || !out || width <= 0 || height <= 0) return SGS_EINVAL;
  if (!(fovx_rad > 0.0 && fovx_rad < M_PI) || !(fovy_rad < M_PI) || !isfinite(near_z))
    return SGS_EINVAL;
  for (int k = 0; k < 16; ++k)
    if (!isfinite(c2w_gl[k])) return SGS_EINVAL;
  // M_cv = M_gl T_align, T_align = diag(1,-1,-1,1): flip the camera's y and z axes
  double A[3][3], p[3];
  for (int r = 0; r < 3; ++r) {
    A[r][0] = c2w_gl[4 * r + 0];
    A[r][1] = -c2w_gl[4 * r + 1];
    A[r][2] = -c2w_gl[4 * r + 2];
    p[r] = c2w_gl[4 * r + 3];
  }
  // w2c = M_cv^-1 = [A^-1 | -A^-1 p]
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  if (!(fabs(det) > 1e-12)) return SGS_EINVAL;
  double I[3][3];
  I[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
  I[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  I[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  I[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
  I[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  I[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  I[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
  I[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  I[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  memset(out, 0, sizeof(*out));
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) out->w2c[4 * r + c] = (float)I[r][c];
    out->w2c[4 * r + 3] = (float)(-(I[r][0] * p[0] + I[r][1] * p[1] + I[r][2] * p[2]));
    out->campos[r] = (float)p[r];
  }
  // K from (W, H, FoV)
  const double fx = width / (2.0 * tan(fovx_rad / 2.0));
  const double fy = fovy_rad > 0.0 ? height / (2.0 * tan(fovy_rad / 2.0)) : fx;
  out->width = width;
  out->height = height;
  out->fx = (float)fx;
  out->fy = (float)fy;
  out->cx = 0.5f * (float)width;
  out->cy = 0.5f * (float)height;
  out->near_z = near_z;
  for (int k = 0; k < 3; ++k) out->bg[k] = bg ? bg[k] : 0.0f;
  return SGS_OK;
}

sgs_status sgs_camera_layout(sgs_camera* cams, int32_t n_views, const sgs_options* opt,
                             int64_t* total_tiles, int64_t* total_pixels) {
  if (!cams || n_views <= 0 || !options_ok(opt)) return SGS_EINVAL;
  int64_t tb = 0, pb = 0;
  for (int v = 0; v < n_views; ++v) {
    sgs_camera& k = cams[v];
    if (k.width <= 0 || k.height <= 0) return SGS_EINVAL;
    k.tiles_x = (k.width + opt->tile_w - 1) / opt->tile_w;
    k.tiles_y = (k.height + opt->tile_h - 1) / opt->tile_h;
    k.tile_base = (int32_t)tb;
    k.pix_base = pb;
    tb += (int64_t)k.tiles_x * k.tiles_y;
    pb += (int64_t)k.width * k.height;
    if (tb >= ((int64_t)1 << 31) || k.tiles_x > 65535 || k.tiles_y > 65535) return SGS_EINVAL;
  }
  if (total_tiles) *total_tiles = tb;
  if (total_pixels) *total_pixels = pb;
  return SGS_OK;
}

int64_t sgs_geom_rec_floats(int64_t m, int32_t enhanced) {
  (void)enhanced;   // records: 16 floats each; gradient planes: at most 4 x 4
  return m * 16;
}

int64_t sgs_geom_block_entries(int64_t n, int32_t n_views) {
  return (int64_t)n_views * ((n + 255) / 256) + 1;
}

// The sort mode a call runs: sort_mode, or with -1 (auto) row binning
// (mode 2) from SGS_AUTO_ROWBIN_CAPACITY instances of capacity up (where it
// measured faster) and the tile-key sort (mode 1) below.
static int32_t sort_mode_for(const sgs_options* opt, int64_t cap) {
  if (opt->sort_mode >= 0) return opt->sort_mode;
  return cap >= SGS_AUTO_ROWBIN_CAPACITY ? 2 : 1;
}

size_t sgs_bin_sort_scratch_bytes(int64_t m, int64_t cap, int64_t total_tiles,
                                  const sgs_options* opt) {
  if (!opt || m < 0 || cap < 0) return 0;
  return sgs::bin_sort_scratch_bytes(m, cap, total_tiles, sort_mode_for(opt, cap));
}

sgs_status sgs_preprocess(const sgs_params* p, const sgs_camera* cams_host,
                          const sgs_camera* cams_dev, int32_t n_views, const sgs_options* opt,
                          const sgs_geom* g, void* stream) {
  if (!params_ok(p) || !cams_ok(cams_host, n_views) || !cams_dev || !options_ok(opt) || !g)
    return SGS_EINVAL;
  if (p->n > 0 && (!g->rec || !g->depth || !g->rect || !g->tiles)) return SGS_EINVAL;
  if (!g->block_off) return SGS_EINVAL;
  if (g->enhanced != (p->opa2_logit != nullptr ? 1 : 0)) return SGS_EINVAL;
  if (p->n * (int64_t)n_views >= ((int64_t)1 << 32)) return SGS_EUNSUPPORTED;
  return sgs::launch_preprocess(p, cams_dev, n_views, opt, g, (hipStream_t)stream);
}

// Sort mode 2 needs the row counts, at most 64 views, 256 tiles per view
// row and 1024 tile rows in all: the number of global tile rows then, else
// 0 (mode 1 sorts; same results).
static int32_t rowbin_rows(const sgs_camera* cams_host, int32_t n_views, bool have_rows) {
  if (!have_rows || n_views > 64) return 0;
  int64_t rows = 0;
  int32_t tx_max = 1;
  for (int v = 0; v < n_views; ++v) {
    rows += cams_host[v].tiles_y;
    tx_max = std::max(tx_max, cams_host[v].tiles_x);
  }
  return rows <= 1024 && tx_max <= 256 ? (int32_t)std::max<int64_t>(rows, 1) : 0;
}

int32_t sgs_bin_sort_mode(const sgs_options* opt, int64_t inst_capacity, const sgs_camera* cams_host,
                          int32_t n_views, int32_t have_rows) {
  if (!options_ok(opt) || !cams_ok(cams_host, n_views) || inst_capacity < 0) return -1;
  const int32_t mode = sort_mode_for(opt, inst_capacity);
  if (mode == 2 && rowbin_rows(cams_host, n_views, have_rows != 0) == 0) return 1;
  return mode;
}

sgs_status sgs_bin_sort(const sgs_geom* g, int64_t m, const sgs_camera* cams_host,
                        const sgs_camera* cams_dev, int32_t n_views, const sgs_options* opt,
                        int64_t inst_capacity, uint64_t* keys, uint32_t* vals,
                        uint32_t* tile_ranges, uint32_t* n_inst_dev, const sgs_schedule* sched,
                        void* scratch, size_t scratch_bytes, void* stream) {
  if (!g || m < 0 || !cams_ok(cams_host, n_views) || !cams_dev || !options_ok(opt) ||
      inst_capacity < 0 || inst_capacity >= ((int64_t)1 << 32) || !tile_ranges || !n_inst_dev)
    return SGS_EINVAL;
  if (m % n_views != 0 || m >= ((int64_t)1 << 32)) return SGS_EINVAL;
  if (inst_capacity > 0 && !vals) return SGS_EINVAL;
  const int32_t mode = sort_mode_for(opt, inst_capacity);
  if (mode == 0 && inst_capacity > 0 && !keys) return SGS_EINVAL;
  if (m > 0 && (!g->rec || !g->depth || !g->rect || !g->tiles || !g->block_off)) return SGS_EINVAL;
  if (g->enhanced != 0 && g->enhanced != 1) return SGS_EINVAL;
  const int64_t tt = tiles_total(cams_host, n_views);
  if (!scratch || scratch_bytes < sgs::bin_sort_scratch_bytes(m, inst_capacity, tt, mode))
    return SGS_ECAPACITY;
  float near_min = cams_host[0].near_z;
  for (int v = 1; v < n_views; ++v) near_min = std::min(near_min, cams_host[v].near_z);
  const int32_t rb_rows = mode == 2 ? rowbin_rows(cams_host, n_views, m == 0 || g->rows) : 0;
  int32_t rb_tx = 1;   // the most tiles per row of any view (sizes the placement's columns)
  for (int v = 0; v < n_views; ++v) rb_tx = std::max(rb_tx, cams_host[v].tiles_x);
  sgs_options o = *opt;
  o.sort_mode = mode;
  return sgs::launch_bin_sort(g, m, m / n_views, cams_dev, n_views, tt, &o, inst_capacity, keys,
                              vals, tile_ranges, n_inst_dev, sched ? sched->tile_order : nullptr,
                              scratch, near_min, rb_rows, rb_tx, (hipStream_t)stream);
}

sgs_status sgs_bin_sort_noalloc(const sgs_geom* g, int64_t m, const sgs_camera* cams_host,
                                const sgs_camera* cams_dev, int32_t n_views,
                                const sgs_options* opt, int64_t inst_capacity, uint64_t* keys,
                                uint32_t* vals, uint32_t* tile_ranges, uint32_t* n_inst_dev,
                                const sgs_schedule* sched, void* stream) {
  // the same checks as sgs_bin_sort, then the size check against the fixed
  // array, before any HIP call that touches it
  if (!g || m < 0 || !cams_ok(cams_host, n_views) || !cams_dev || !options_ok(opt) ||
      inst_capacity < 0 || inst_capacity >= ((int64_t)1 << 32))
    return SGS_EINVAL;
  const size_t need = sgs::bin_sort_scratch_bytes(m, inst_capacity, tiles_total(cams_host, n_views),
                                                  sort_mode_for(opt, inst_capacity));
  if (need > (size_t)SGS_NOALLOC_SCRATCH_BYTES) return SGS_ECAPACITY;
  void* ws = nullptr;
  const sgs_status st = noalloc_scratch(&ws);
  if (st != SGS_OK) return st;
  return sgs_bin_sort(g, m, cams_host, cams_dev, n_views, opt, inst_capacity, keys, vals,
                      tile_ranges, n_inst_dev, sched, ws, (size_t)SGS_NOALLOC_SCRATCH_BYTES, stream);
}

sgs_status sgs_render_fwd(const sgs_geom* g, int64_t m, const uint32_t* vals,
                          int64_t inst_capacity, const uint32_t* tile_ranges,
                          const sgs_schedule* sched, const sgs_camera* cams_host,
                          const sgs_camera* cams_dev, int32_t n_views, int32_t enhanced,
                          const sgs_options* opt, float* out_rgb, float* out_T,
                          uint32_t* out_last, uint32_t* out_count, uint32_t* out_eval,
                          int64_t total_pixels, void* stream) {
  if (!g || (m > 0 && !g->rec) || m < 0 || !tile_ranges || !cams_ok(cams_host, n_views) ||
      !cams_dev || !options_ok(opt) || !out_rgb || !out_T || !out_last)
    return SGS_EINVAL;
  if (total_pixels != pixels_total(cams_host, n_views)) return SGS_EINVAL;
  if (inst_capacity < 0 || inst_capacity >= ((int64_t)1 << 32) || (!vals && inst_capacity > 0))
    return SGS_EINVAL;
  if ((enhanced ? 1 : 0) != g->enhanced) return SGS_EINVAL;
  return sgs::launch_blend_fwd(g, m, vals, inst_capacity, tile_ranges, sched, cams_dev, n_views,
                               tiles_total(cams_host, n_views), enhanced ? 1 : 0, opt, out_rgb,
                               out_T, out_last, out_count, out_eval, total_pixels, (hipStream_t)stream);
}

sgs_status sgs_render_bwd(const sgs_params* p, const sgs_geom* g, int64_t m,
                          const uint32_t* vals, int64_t inst_capacity,
                          const uint32_t* tile_ranges, const sgs_schedule* sched,
                          const sgs_camera* cams_host, const sgs_camera* cams_dev,
                          int32_t n_views, const sgs_options* opt, const float* out_T,
                          const uint32_t* out_last, const float* dL_drgb, int64_t total_pixels,
                          const sgs_geom_grad* g2d, const sgs_params_grad* grad, void* stream) {
  if (!params_ok(p) || !g || !tile_ranges || !cams_ok(cams_host, n_views) || !cams_dev ||
      !options_ok(opt) || !out_T || !out_last || !dL_drgb || !g2d || !grad)
    return SGS_EINVAL;
  if (m > 0 && (!g->rec || !g->tiles || !g2d->rec))
    return SGS_EINVAL;
  if (m != p->n * (int64_t)n_views) return SGS_EINVAL;
  if (total_pixels != pixels_total(cams_host, n_views)) return SGS_EINVAL;
  if (inst_capacity < 0 || inst_capacity >= ((int64_t)1 << 32) || (!vals && inst_capacity > 0))
    return SGS_EINVAL;
  const int enhanced = p->opa2_logit != nullptr;
  if (enhanced != g->enhanced) return SGS_EINVAL;
  sgs_status st = sgs::launch_blend_bwd(g, m, vals, inst_capacity, tile_ranges, sched, cams_dev,
                                        n_views,
                                        tiles_total(cams_host, n_views), enhanced, opt, out_T,
                                        out_last, dL_drgb, total_pixels, g2d->rec,
                                        (hipStream_t)stream);
  if (st != SGS_OK) return st;
  return sgs::launch_preprocess_bwd(p, cams_dev, n_views, opt, g, g2d->rec, grad,
                                    (hipStream_t)stream);
}

void sgs_default_densify_options(sgs_densify_options* o) {
  if (!o) return;
  o->tau_uv = 0.001f;
  o->tau_z = 0.001f;
  o->dense_scale = 0.01f;
  o->split_shrink = 1.6f;
}

int64_t sgs_densify_scratch_words(int64_t n) {
  return n < 0 ? 0 : (n + 255) / 256 + 1;
}

sgs_status sgs_densify(const sgs_params* p, const float* uv_sum, const uint32_t* view_count,
                       const float* z_max, const sgs_densify_options* opt, uint8_t* decision,
                       const sgs_densify_out* out, uint32_t* n_out_dev, uint32_t* scratch,
                       void* stream) {
  if (!params_ok(p) || !opt || !out || !n_out_dev || !scratch) return SGS_EINVAL;
  if ((uv_sum == nullptr) != (view_count == nullptr)) return SGS_EINVAL;
  if (p->n > 0 && !decision) return SGS_EINVAL;
  if (!(isfinite(opt->tau_uv) && isfinite(opt->tau_z) && opt->dense_scale > 0.0f &&
        isfinite(opt->dense_scale) && opt->split_shrink > 1.0f && isfinite(opt->split_shrink)))
    return SGS_EINVAL;
  if (out->capacity < 0) return SGS_EINVAL;
  if (out->capacity > 0 &&
      (!out->mean || !out->log_scale || !out->quat || !out->opa_logit || !out->sh ||
       (p->skew && !out->skew) || (p->opa2_logit && !out->opa2_logit) ||
       (p->opa_dir && !out->opa_dir)))
    return SGS_EINVAL;
  if (2 * p->n >= ((int64_t)1 << 32)) return SGS_EUNSUPPORTED;
  return sgs::launch_densify(p, uv_sum, view_count, z_max, opt, decision, scratch, out, n_out_dev,
                             (hipStream_t)stream);
}

sgs_status sgs_adam_step(const sgs_adam_group* groups, int32_t n_groups, float* state,
                         float beta1, float beta2, float eps, void* stream) {
  if (!groups || !state || n_groups <= 0 || n_groups > SGS_ADAM_MAX_GROUPS) return SGS_EINVAL;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return SGS_EINVAL;
  for (int k = 0; k < n_groups; ++k) {
    const sgs_adam_group& g = groups[k];
    if (g.n < 0 || !isfinite(g.lr)) return SGS_EINVAL;
    if (g.n > 0 && (!g.param || !g.grad || !g.m1 || !g.m2)) return SGS_EINVAL;
  }
  return sgs::launch_adam(groups, n_groups, state, beta1, beta2, eps, (hipStream_t)stream);
}

}  // extern "C"
