// Per-tile compositing of projected skew Gaussians, forward and backward.
//
// One workgroup per screen tile (TW x TH pixels, one pixel per thread, each
// wave64 owns an 8x8 block of the tile).  The tile's sorted list is walked in
// batches of B records staged in LDS.  When a batch is staged, each record
// gets a mask of the 8x8 wave blocks its evaluation ellipse (the region where
// the pair is not skipped by the exponent test) can touch, and each wave gets
// its own compacted, order-preserving list of record indices; a wave only
// visits its own list.  This is exact: a record missing from a wave's list
// would have failed the skip test on every lane of that wave.  All lanes of a
// wave read the same record at the same time, so per-record branches (a
// symmetric record skips erf) never diverge.
//
// Forward (Alg. 1): alpha = min(alpha_max, d G' (1 + erf z)) per pair, pairs
// below alpha_min skipped, a pixel stops before T would drop below t_min,
// C += c alpha T.  Backward (Alg. 2): each pixel walks its list from its last
// contributor to the front, rebuilding T_k = T_{k+1} / (1 - alpha_k) from the
// final transmittance (nothing per pair is stored), with the colour behind k
// kept as a running sum.  Per-pair partial derivatives are summed over each
// 16-lane row with a transposing DPP sum (afterwards each lane holds one of
// the record's row sums), over rows and waves with LDS atomics, and written
// with one set of global atomics per (record, tile).  Pairs are evaluated in
// base 2 from per-record constants folded in when a batch is staged.
#include <algorithm>

#include "sgs_dev.h"

namespace sgs {

struct BlendArgs {
  const float4* rec;       // [M][4] record slots
  const uint32_t* vals;
  const uint2* ranges;
  const sgs_camera* cams;
  int32_t n_views;
  int32_t total_tiles;
  uint32_t n_vals;         // length of vals (instance capacity)
  uint32_t m;              // number of records
  float alpha_min, alpha_max, t_min;
  int64_t P;               // pixels of all views (plane stride)
  float* out_rgb;
  float* out_T;
  uint32_t* out_last;
  uint32_t* out_count;     // optional: contributing pairs per pixel
  uint32_t* out_eval;      // optional: evaluated pairs per pixel (past the exponent test)
  const uint32_t* tile_order;  // optional: tiles in this order (longest lists first)
  uint32_t* work_counter;      // optional: persistent workgroups take tiles from it
  int32_t n_quad;              // forward: the first n_quad tiles of tile_order run split
  bool quarter_lists;          // forward: tiles walk quarter lists (fwd_tile_q)
  // backward
  const float* cT;
  const uint32_t* clast;
  const float* dL;
  float4* g0;
  float4* g1;
  float4* g2;
  float4* g3;
};

struct TileSetup {
  int tile, view;
  int px, py;      // this thread's pixel
  int ox, oy;      // tile origin in pixels
  int gx, gy;      // origin of the grid of wave blocks
  bool inside;
  const sgs_camera* cam;
};

template <int TW, int TH>
__device__ __forceinline__ bool setup_tile(const BlendArgs& a, int tile, TileSetup& s) {
  s.tile = tile;
  if (tile < 0 || tile >= a.total_tiles) return false;
  s.view = find_view(a.cams, a.n_views, s.tile);
  s.cam = a.cams + s.view;
  const int lt = s.tile - s.cam->tile_base;
  const int tx = lt % s.cam->tiles_x, ty = lt / s.cam->tiles_x;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  s.ox = tx * TW;
  s.oy = ty * TH;
  s.gx = s.ox;
  s.gy = s.oy;
  s.px = s.ox + (w % (TW / 8)) * 8 + (l & 7);
  s.py = s.oy + (w / (TW / 8)) * 8 + (l >> 3);
  s.inside = s.px < s.cam->width && s.py < s.cam->height;
  return true;
}

// List entries: the record's slot in the batch, LIST_SKEW set when its 2D
// skew is nonzero (NaN counting as nonzero); mask bit SKEW_BIT carries the
// same flag while the lists are built.
constexpr uint32_t LIST_SLOT = 0xffu, LIST_SKEW = 0x100u, SKEW_BIT = 0x80u;

// Staged batch of B records and the compacted lists: NL = NW lists, one per
// wave, or NL = 4 NW, one per 4x4 quarter of each wave's 8x8 block (the
// forward tile path, whose per-record quarter masks are kept per row of
// wave blocks in qm).
template <int TW, int TH, int B, bool ENH, int NL = TW * TH / 64>
struct Stage {
  static constexpr int NT = TW * TH;
  static constexpr int NW = NT / 64;
  static constexpr int NG = B / 64;   // 64-record groups of the batch
  static constexpr bool QL = NL > NW;
  // r0 = (mu_x, mu_y, A, B), r1 = (C, bxs, bys, D), r2 = (r, g, b, log2 e
  // log_thr + D): the base-2 constants of pair_log2 / pair_eval2
  float4 r0[B], r1[B], r2[B];
  float4 r3[ENH ? B : 1];
  float idv[B];           // 1/d (backward)
  uint32_t rid[B];
  uint8_t mask[B];
  uint8_t qm[QL ? TH / 8 : 1][QL ? B : 1];
  uint16_t cnt[NL][NG];
  uint16_t list[NL][B];
  uint16_t n[NL];
};

// x-range [xl, xr] (delta coordinates) of the ellipse {delta : delta^T Q
// delta <= R2}, Q = [[a, b], [b, c]] positive definite, over the band of
// rows u in [u0, u1], widened by the margins of the tile extent; false if
// the band misses the ellipse.  On a row u the ellipse spans
// x = (-b u +- sqrt(a R2 - det u^2)) / a; over the band the extremes are at
// the band's ends or where the ellipse's own x extremes lie (u = +-yx).
// Approximate sqrt and reciprocal: their error is far inside the margins.
__device__ __forceinline__ bool band_xrange(float a, float b, float c, float det, float R2,
                                            float u0, float u1, float& xl, float& xr) {
  const float ia = __builtin_amdgcn_rcpf(a);
  const float idet = __builtin_amdgcn_rcpf(det);
  const float ey = __builtin_amdgcn_sqrtf(R2 * a * idet);
  u0 = fmaxf(u0, -ey);
  u1 = fminf(u1, ey);
  if (!(u0 <= u1)) return false;
  const float aR2 = a * R2;
  const float r0 = __builtin_amdgcn_sqrtf(fmaxf(aR2 - det * u0 * u0, 0.0f));
  const float r1 = __builtin_amdgcn_sqrtf(fmaxf(aR2 - det * u1 * u1, 0.0f));
  xr = fmaxf((-b * u0 + r0) * ia, (-b * u1 + r1) * ia);
  xl = fminf((-b * u0 - r0) * ia, (-b * u1 - r1) * ia);
  const float ex = __builtin_amdgcn_sqrtf(R2 * c * idet);          // the ellipse's largest x
  const float yx = -b * ex * __builtin_amdgcn_rcpf(c);             // ... reached at dy = yx
  if (yx >= u0 && yx <= u1) xr = ex;
  if (-yx >= u0 && -yx <= u1) xl = -ex;
  // widen outwards on both sides: 0.1% of the offset plus 0.01 px
  xr = xr + (fabsf(xr) * 1e-3f + 0.01f);
  xl = xl - (fabsf(xl) * 1e-3f + 0.01f);
  return true;
}

// Loads records [idx0, idx0 + cnt) of the tile list into the stage and builds
// the per-wave lists.  Wave w owns the BS x BS pixel block at
// (gx, gy) + BS * (w % GW, w / GW): 8x8 blocks covering the tile (GW = TW/8),
// or 4x4 blocks covering an 8x8 quarter (GW = 2).  Every thread of the block
// must call it.
template <int TW, int TH, int B, bool ENH, int BS = 8, int NL>
__device__ __forceinline__ void stage_batch(const BlendArgs& a, const TileSetup& ts, uint32_t idx0,
                                            int cnt, Stage<TW, TH, B, ENH, NL>& S) {
  constexpr int GW = BS == 8 ? TW / 8 : 2;
  constexpr float EXT = (float)(BS - 1);      // pixel-centre span of a block
  constexpr float HALF = 0.5f * EXT;
  using St = Stage<TW, TH, B, ENH, NL>;
  const int t = threadIdx.x, lane = t & 63;
  const uint64_t lt = lanemask_lt();
  for (int k = t; k < B; k += St::NT) {
    uint32_t msk = 0;
    if (k < cnt) {
      uint32_t m = a.vals[idx0 + k];
      if (m >= a.m) m = 0;
      const float4* rp = a.rec + 4 * (uint64_t)m;
      const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2];
      S.rid[k] = m;
      const float D = __builtin_amdgcn_logf(q1.w);   // log2 d
      S.r0[k] = make_float4(q0.x, q0.y, SGS_KA * q0.z, -SGS_L2E * q0.w);
      S.r1[k] = make_float4(SGS_KA * q1.x, SGS_KZ * q1.y, SGS_KZ * q1.z, D);
      S.r2[k] = make_float4(q2.x, q2.y, q2.z, fmaf(SGS_L2E, q2.w, D));
      S.idv[k] = 1.0f / q1.w;
      if (ENH) S.r3[k] = rp[3];
      if ((q1.y != 0.0f) || (q1.z != 0.0f)) msk = SKEW_BIT;
      // the ellipse delta^T Q delta <= -2 log_thr outside which every pair
      // is skipped, with the margins of the tile extent
      const float det = q0.z * q1.x - q0.w * q0.w;
      const float R2 = -2.0f * q2.w * 1.002f + 1e-3f;
      if (!(det > 0.0f) || !(q0.z > 0.0f) || !(R2 > 0.0f) || !(R2 < 1e30f) || !(det < 1e30f)) {
        msk |= (1u << St::NW) - 1u;
      } else {
        // skew half-plane: alpha <= d (1 + erf(z)) stays below alpha_min
        // wherever beta.delta < sqrt2 * zcut
        const bool skew = (q1.y != 0.0f) || (q1.z != 0.0f);
        const float zc = skew ? skew_zcut(a.alpha_min, q1.w) : -1e30f;
        const float need = zc * 1.41421356f;
        // the ellipse's x-range over each row of wave blocks
        constexpr int GR = St::NW / GW;
        float bxl[GR], bxr[GR];
        bool bok[GR];
#pragma unroll
        for (int r = 0; r < GR; ++r) {
          const float ly = (float)(ts.gy + r * BS) + 0.5f;
          bok[r] = band_xrange(q0.z, q0.w, q1.x, det, R2, ly - q0.y - 0.01f, ly + EXT - q0.y + 0.01f,
                               bxl[r], bxr[r]);
        }
#pragma unroll
        for (int w = 0; w < St::NW; ++w) {
          const float lx = (float)(ts.gx + (w % GW) * BS) + 0.5f;
          const float ly = (float)(ts.gy + (w / GW) * BS) + 0.5f;
          const int r = w / GW;
          bool hit = bok[r] && bxr[r] >= lx - q0.x && bxl[r] <= lx + EXT - q0.x;
          if (hit && zc > -1e29f) {
            const float top = skew_box_max(q1.y, q1.z, lx + HALF, ly + HALF, q0.x, q0.y, HALF, HALF);
            hit = top + 1e-3f * (1.0f + fabsf(top) + fabsf(need)) >= need;
          }
          if (hit) msk |= 1u << w;
        }
      }
    }
    S.mask[k] = (uint8_t)msk;
#pragma unroll
    for (int w = 0; w < St::NW; ++w) {
      const uint64_t bal = __ballot((msk >> w) & 1u);
      if (lane == 0) S.cnt[w][k >> 6] = (uint16_t)__popcll(bal);
    }
  }
  __syncthreads();
  for (int k = t; k < B; k += St::NT) {
    const uint32_t msk = S.mask[k];
#pragma unroll
    for (int w = 0; w < St::NW; ++w) {
      const bool bit = (msk >> w) & 1u;
      const uint64_t bal = __ballot(bit);
      if (bit) {
        uint32_t off = (uint32_t)__popcll(bal & lt);
        for (int g = 0; g < (k >> 6); ++g) off += S.cnt[w][g];
        S.list[w][off] = (uint16_t)(k | ((msk & SKEW_BIT) ? LIST_SKEW : 0u));
      }
    }
  }
  if (t < St::NW) {
    uint32_t s = 0;
    for (int g = 0; g < St::NG; ++g) s += S.cnt[t][g];
    S.n[t] = (uint16_t)s;
  }
  __syncthreads();
}

// Loads records [idx0, idx0 + cnt) and builds the quarter lists: list 4 w + q
// holds the records whose extent reaches the 4x4 block at (gx, gy) +
// (8 (w % GW) + 4 (q & 1), 8 (w / GW) + 4 (q >> 1)), the quarters of wave w's
// 8x8 block.  A record is tested by TH / 8 threads, one per row of wave
// blocks (two 4-pixel bands each); the first of them stages its constants.
// Same tests as stage_batch with 4x4 blocks.  Every thread must call it.
template <int TW, int TH, int B, bool ENH, int NL>
__device__ __forceinline__ void stage_batch_q(const BlendArgs& a, const TileSetup& ts, uint32_t idx0,
                                              int cnt, Stage<TW, TH, B, ENH, NL>& S) {
  using St = Stage<TW, TH, B, ENH, NL>;
  static_assert(NL == 4 * St::NW && (B & (B - 1)) == 0 && B >= 64, "quarter lists of a power-of-two batch");
  constexpr int GW = TW / 8, WR = TH / 8;
  constexpr int QB = 4 * GW;                   // lists per row of wave blocks
  const int t = threadIdx.x, lane = t & 63;
  const uint64_t lt = lanemask_lt();
  // (B and NT are multiples of 64: the 64 items of a wave share one row)
  for (int it = t; it < B * WR; it += St::NT) {
    const int k = it & (B - 1), wr = it / B;
    uint32_t msk = 0;
    if (k < cnt) {
      uint32_t m = a.vals[idx0 + k];
      if (m >= a.m) m = 0;
      const float4* rp = a.rec + 4 * (uint64_t)m;
      const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2];
      const bool skew = (q1.y != 0.0f) || (q1.z != 0.0f);
      if (wr == 0) {
        S.rid[k] = m;
        const float D = __builtin_amdgcn_logf(q1.w);   // log2 d
        S.r0[k] = make_float4(q0.x, q0.y, SGS_KA * q0.z, -SGS_L2E * q0.w);
        S.r1[k] = make_float4(SGS_KA * q1.x, SGS_KZ * q1.y, SGS_KZ * q1.z, D);
        S.r2[k] = make_float4(q2.x, q2.y, q2.z, fmaf(SGS_L2E, q2.w, D));
        S.idv[k] = 1.0f / q1.w;
        if (ENH) S.r3[k] = rp[3];
        S.mask[k] = skew ? (uint8_t)SKEW_BIT : (uint8_t)0;
      }
      const float det = q0.z * q1.x - q0.w * q0.w;
      const float R2 = -2.0f * q2.w * 1.002f + 1e-3f;
      if (!(det > 0.0f) || !(q0.z > 0.0f) || !(R2 > 0.0f) || !(R2 < 1e30f) || !(det < 1e30f)) {
        msk = (1u << QB) - 1u;
      } else {
        const float zc = skew ? skew_zcut(a.alpha_min, q1.w) : -1e30f;
        const float need = zc * 1.41421356f;
        float bxl[2], bxr[2];
        bool bok[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const float ly = (float)(ts.gy + (2 * wr + r) * 4) + 0.5f;
          bok[r] = band_xrange(q0.z, q0.w, q1.x, det, R2, ly - q0.y - 0.01f, ly + 3.0f - q0.y + 0.01f,
                               bxl[r], bxr[r]);
        }
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          const int r = (b >> 1) & 1;                                  // band of quarter b & 3
          const float lx = (float)(ts.gx + (b >> 2) * 8 + (b & 1) * 4) + 0.5f;
          const float ly = (float)(ts.gy + (2 * wr + r) * 4) + 0.5f;
          bool hit = bok[r] && bxr[r] >= lx - q0.x && bxl[r] <= lx + 3.0f - q0.x;
          if (hit && zc > -1e29f) {
            const float top = skew_box_max(q1.y, q1.z, lx + 1.5f, ly + 1.5f, q0.x, q0.y, 1.5f, 1.5f);
            hit = top + 1e-3f * (1.0f + fabsf(top) + fabsf(need)) >= need;
          }
          if (hit) msk |= 1u << b;
        }
      }
    } else if (wr == 0) {
      S.mask[k] = 0;
    }
    S.qm[wr][k] = (uint8_t)msk;
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      const uint64_t bal = __ballot((msk >> b) & 1u);
      if (lane == 0) S.cnt[wr * QB + b][k >> 6] = (uint16_t)__popcll(bal);
    }
  }
  __syncthreads();
  for (int it = t; it < B * WR; it += St::NT) {
    const int k = it & (B - 1), wr = it / B;
    const uint32_t msk = S.qm[wr][k];
    const uint32_t sk = (S.mask[k] & SKEW_BIT) ? LIST_SKEW : 0u;
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      const bool bit = (msk >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      if (bit) {
        const int l = wr * QB + b;
        uint32_t off = (uint32_t)__popcll(bal & lt);
        for (int g = 0; g < (k >> 6); ++g) off += S.cnt[l][g];
        S.list[l][off] = (uint16_t)(k | sk);
      }
    }
  }
  if (t < NL) {
    uint32_t s = 0;
    for (int g = 0; g < St::NG; ++g) s += S.cnt[t][g];
    S.n[t] = (uint16_t)s;
  }
  __syncthreads();
}

// Tile of a one-workgroup-per-tile launch: the given order, else XCD bands.
// (Forward with split tiles: the first 4 * n_quad workgroups run the quarters
// of the first n_quad tiles of the order; the rest take the following ones.)
__device__ __forceinline__ int launch_tile(const BlendArgs& a) {
  if (a.tile_order) {
    const uint32_t idx = blockIdx.x - 3u * (uint32_t)a.n_quad;
    return idx < (uint32_t)a.total_tiles ? (int)a.tile_order[idx] : a.total_tiles;
  }
  return xcd_tile(blockIdx.x, a.total_tiles, gridDim.x);
}

// Persistent workgroups: the next tile index from the counter (every
// workgroup ends once the counter passes the number of tiles).
__device__ __forceinline__ int next_tile(const BlendArgs& a, uint32_t* s_next) {
  if (threadIdx.x == 0) *s_next = atomicAdd(a.work_counter, 1u);
  __syncthreads();
  const uint32_t idx = *s_next;
  __syncthreads();
  if (idx >= (uint32_t)a.total_tiles) return -1;
  return a.tile_order ? (int)a.tile_order[idx] : (int)idx;
}

template <int TW, int TH, int B, bool ENH, bool CNT, int NL>
__device__ __forceinline__ void fwd_tile(const BlendArgs& a, int tile, Stage<TW, TH, B, ENH, NL>& S) {
  TileSetup ts;
  if (!setup_tile<TW, TH>(a, tile, ts)) return;
  const int w = threadIdx.x >> 6;
  const float fx = (float)ts.px + 0.5f, fy = (float)ts.py + 0.5f;
  uint2 rg = a.ranges[ts.tile];
  rg.y = min(rg.y, a.n_vals);
  rg.x = min(rg.x, rg.y);
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last = 0, count = 0, evals = 0;
  bool done = !ts.inside;
  for (uint32_t base = rg.x; base < rg.y; base += B) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)B, rg.y - base);
    stage_batch<TW, TH, B, ENH>(a, ts, base, cnt, S);
    // the wave walks its list together: control flow is wave-uniform, lanes
    // that are finished or outside a record's ellipse are masked
    const int nw = __builtin_amdgcn_readfirstlane(S.n[w]);   // wave-uniform
    int jn = nw > 0 ? S.list[w][0] : 0;
    // (a guarded body and a wave-uniform exit flag in the loop condition,
    // rather than continue and break)
    bool ended = false;
    for (int i = 0; i < nw && !ended; ++i) {
      const uint32_t e = (uint32_t)__builtin_amdgcn_readfirstlane(jn);
      const int j = (int)(e & LIST_SLOT);
      if (i + 1 < nw) jn = S.list[w][i + 1];
      const float4 r0 = S.r0[j];
      const float4 r1 = S.r1[j];
      const float4 r2 = S.r2[j];
      const float dx = fx - r0.x, dy = fy - r0.y;
      const float l2 = pair_log2(r0.z, r0.w, r1.x, r1.w, dx, dy);
      const bool in = !done && l2 >= r2.w;
      if (wave_any(in)) {
        if (CNT && in) ++evals;
        Pair2 p;
        pair_eval2(l2, r1.y, r1.z, dx, dy, (e & LIST_SKEW) != 0u, p);
        float at = p.at;
        if (ENH) {
          const float4 r3 = S.r3[j];
          float eu, ee;
          at *= enh_opacity(r3.x, r3.y, r3.z, r3.w, dx, dy, eu, ee);
        }
        const float alpha = fminf(a.alpha_max, at);
        // the skip test again rather than `in`: a bool kept across the branch
        // above costs two VALU instructions to rebuild as a lane mask
        const bool take = !done && l2 >= r2.w && alpha >= a.alpha_min;
        const float Tn = T * (1.0f - alpha);
        const bool stop = take && Tn < a.t_min;
        if (take && !stop) {
          const float wgt = alpha * T;
          C0 = fmaf(r2.x, wgt, C0);
          C1 = fmaf(r2.y, wgt, C1);
          C2 = fmaf(r2.z, wgt, C2);
          T = Tn;
          last = base - rg.x + (uint32_t)j + 1u;
          if (CNT) ++count;
        }
        done = done || stop;
        ended = wave_any(stop) && wave_all(done);
      }
    }
  }
  if (ts.inside) {
    const int64_t pix = ts.cam->pix_base + (int64_t)ts.py * ts.cam->width + ts.px;
    a.out_rgb[pix] = fmaf(T, ts.cam->bg[0], C0);
    a.out_rgb[a.P + pix] = fmaf(T, ts.cam->bg[1], C1);
    a.out_rgb[2 * a.P + pix] = fmaf(T, ts.cam->bg[2], C2);
    a.out_T[pix] = T;
    a.out_last[pix] = last;
    if (CNT) {
      if (a.out_count) a.out_count[pix] = count;
      if (a.out_eval) a.out_eval[pix] = evals;
    }
  }
}

// The same with quarter lists: wave w walks lists 4 w .. 4 w + 3 together,
// entry i of each at step i, each lane in its own quarter's list, so a
// record costs a step only in the quarters its extent reaches.  Every pixel
// takes the same records in the same order: identical results.
template <int TW, int TH, int B, bool ENH, bool CNT, int NL>
__device__ __forceinline__ void fwd_tile_q(const BlendArgs& a, int tile, Stage<TW, TH, B, ENH, NL>& S) {
  static_assert(NL == 4 * (TW * TH / 64), "quarter lists");
  TileSetup ts;
  if (!setup_tile<TW, TH>(a, tile, ts)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the lane's pixel is (lane & 7, lane >> 3) of the wave's 8x8 block: its
  // 4x4 quarter and that quarter's list
  const int ql = 4 * w + (((lane >> 5) << 1) | ((lane >> 2) & 1));
  const float fx = (float)ts.px + 0.5f, fy = (float)ts.py + 0.5f;
  uint2 rg = a.ranges[ts.tile];
  rg.y = min(rg.y, a.n_vals);
  rg.x = min(rg.x, rg.y);
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last = 0, count = 0, evals = 0;
  bool done = !ts.inside;
  for (uint32_t base = rg.x; base < rg.y; base += B) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)B, rg.y - base);
    stage_batch_q<TW, TH, B, ENH>(a, ts, base, cnt, S);
    // the wave walks its four quarter lists together, entry i of each at
    // step i: control flow is wave-uniform, lanes that are finished, past
    // their list's end or outside a record's ellipse are masked
    const int nq = S.n[ql];
    const int nw = max(max(__builtin_amdgcn_readlane(nq, 0), __builtin_amdgcn_readlane(nq, 4)),
                       max(__builtin_amdgcn_readlane(nq, 32), __builtin_amdgcn_readlane(nq, 36)));
    int jn = S.list[ql][0];
    // (a guarded body and a wave-uniform exit flag in the loop condition,
    // rather than continue and break)
    bool ended = false;
    for (int i = 0; i < nw && !ended; ++i) {
      const uint32_t e = (uint32_t)jn;
      // (entries past a list's end are stale: masked to a slot in range and
      // never taken)
      const int j = (int)(e & (uint32_t)(B - 1));
      const bool has = i < nq;
      jn = S.list[ql][min(i + 1, B - 1)];
      const float4 r0 = S.r0[j];
      const float4 r1 = S.r1[j];
      const float4 r2 = S.r2[j];
      const float dx = fx - r0.x, dy = fy - r0.y;
      const float l2 = pair_log2(r0.z, r0.w, r1.x, r1.w, dx, dy);
      const bool in = has && !done && l2 >= r2.w;
      if (wave_any(in)) {
        if (CNT && in) ++evals;
        Pair2 p;
        pair_eval2(l2, r1.y, r1.z, dx, dy, (e & LIST_SKEW) != 0u, p);
        float at = p.at;
        if (ENH) {
          const float4 r3 = S.r3[j];
          float eu, ee;
          at *= enh_opacity(r3.x, r3.y, r3.z, r3.w, dx, dy, eu, ee);
        }
        const float alpha = fminf(a.alpha_max, at);
        // the skip test again rather than `in`: a bool kept across the branch
        // above costs two VALU instructions to rebuild as a lane mask
        const bool take = has && !done && l2 >= r2.w && alpha >= a.alpha_min;
        const float Tn = T * (1.0f - alpha);
        const bool stop = take && Tn < a.t_min;
        if (take && !stop) {
          const float wgt = alpha * T;
          C0 = fmaf(r2.x, wgt, C0);
          C1 = fmaf(r2.y, wgt, C1);
          C2 = fmaf(r2.z, wgt, C2);
          T = Tn;
          last = base - rg.x + (uint32_t)j + 1u;
          if (CNT) ++count;
        }
        done = done || stop;
        ended = wave_any(stop) && wave_all(done);
      }
    }
  }
  if (ts.inside) {
    const int64_t pix = ts.cam->pix_base + (int64_t)ts.py * ts.cam->width + ts.px;
    a.out_rgb[pix] = fmaf(T, ts.cam->bg[0], C0);
    a.out_rgb[a.P + pix] = fmaf(T, ts.cam->bg[1], C1);
    a.out_rgb[2 * a.P + pix] = fmaf(T, ts.cam->bg[2], C2);
    a.out_T[pix] = T;
    a.out_last[pix] = last;
    if (CNT) {
      if (a.out_count) a.out_count[pix] = count;
      if (a.out_eval) a.out_eval[pix] = evals;
    }
  }
}

// Value of lane 4*(lane/4) + S (the same quad) in every lane of the quad.
template <int S>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), S * 0x55, 0xf, 0xf, false));
}
template <int S>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, S * 0x55, 0xf, 0xf, false);
}

// Forward of one 8x8 quarter of a 16x16 tile with four lanes per pixel: wave
// w owns a 4x4 block; per round the four lanes of a pixel evaluate four
// consecutive records of the wave's list (one each), then every lane of the
// quad composites the four in list order.  Same decisions and the same
// floating-point operations in the same order as fwd_tile: identical results.
template <int B, bool ENH, bool CNT, int NL>
__device__ __forceinline__ void fwd_quad(const BlendArgs& a, int tile, int quarter,
                                         Stage<16, 16, B, ENH, NL>& S) {
  TileSetup ts;
  if (!setup_tile<16, 16>(a, tile, ts)) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, sub = lane & 3, pq = lane >> 2;
  ts.gx = ts.ox + (quarter & 1) * 8;
  ts.gy = ts.oy + (quarter >> 1) * 8;
  ts.px = ts.gx + (w & 1) * 4 + (pq & 3);
  ts.py = ts.gy + (w >> 1) * 4 + (pq >> 2);
  ts.inside = ts.px < ts.cam->width && ts.py < ts.cam->height;
  const float fx = (float)ts.px + 0.5f, fy = (float)ts.py + 0.5f;
  uint2 rg = a.ranges[ts.tile];
  rg.y = min(rg.y, a.n_vals);
  rg.x = min(rg.x, rg.y);
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last = 0, count = 0, evals = 0;
  bool done = !ts.inside;
  for (uint32_t base = rg.x; base < rg.y; base += B) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)B, rg.y - base);
    stage_batch<16, 16, B, ENH, 4>(a, ts, base, cnt, S);
    const int nw = __builtin_amdgcn_readfirstlane(S.n[w]);   // wave-uniform
    bool ended = false;   // (a wave-uniform exit flag rather than a break)
    for (int i = 0; i < nw && !ended; i += 4) {
      const int k = i + sub;
      const bool has = k < nw;
      const uint32_t e = has ? S.list[w][k] : 0u;
      const int j = (int)(e & LIST_SLOT);
      const float4 r0 = S.r0[j];
      const float4 r1 = S.r1[j];
      const float4 r2 = S.r2[j];
      const float dx = fx - r0.x, dy = fy - r0.y;
      const float l2 = pair_log2(r0.z, r0.w, r1.x, r1.w, dx, dy);
      const bool in = has && !done && l2 >= r2.w;
      float alpha = 0.0f;
      if (CNT && in) ++evals;
      if (wave_any(in)) {
        Pair2 p;
        pair_eval2(l2, r1.y, r1.z, dx, dy, (e & LIST_SKEW) != 0u, p);
        float at = p.at;
        if (ENH) {
          const float4 r3 = S.r3[j];
          float eu, ee;
          at *= enh_opacity(r3.x, r3.y, r3.z, r3.w, dx, dy, eu, ee);
        }
        alpha = fminf(a.alpha_max, at);
      }
      const int take = (in && alpha >= a.alpha_min) ? 1 : 0;
      const int jj = j;
      const float cr = r2.x, cg = r2.y, cb = r2.z;
#define SGS_QUAD_STEP(Q)                                                     \
      {                                                                      \
        const float al = quad_bcast<Q>(alpha);                               \
        if (quad_bcast<Q>(take) && !done) {                                  \
          const float Tn = T * (1.0f - al);                                  \
          if (Tn < a.t_min) {                                                \
            done = true;                                                     \
          } else {                                                           \
            const float wgt = al * T;                                        \
            C0 = fmaf(quad_bcast<Q>(cr), wgt, C0);                           \
            C1 = fmaf(quad_bcast<Q>(cg), wgt, C1);                           \
            C2 = fmaf(quad_bcast<Q>(cb), wgt, C2);                           \
            T = Tn;                                                          \
            last = base - rg.x + (uint32_t)quad_bcast<Q>(jj) + 1u;           \
            if (CNT) ++count;                                                \
          }                                                                  \
        }                                                                    \
      }
      SGS_QUAD_STEP(0)
      SGS_QUAD_STEP(1)
      SGS_QUAD_STEP(2)
      SGS_QUAD_STEP(3)
#undef SGS_QUAD_STEP
      ended = wave_all(done);
    }
  }
  if (CNT)   // the quad's four lanes evaluated disjoint records of the pixel
    evals = (uint32_t)(quad_bcast<0>((int)evals) + quad_bcast<1>((int)evals) + quad_bcast<2>((int)evals) +
                       quad_bcast<3>((int)evals));
  if (ts.inside && sub == 0) {
    const int64_t pix = ts.cam->pix_base + (int64_t)ts.py * ts.cam->width + ts.px;
    a.out_rgb[pix] = fmaf(T, ts.cam->bg[0], C0);
    a.out_rgb[a.P + pix] = fmaf(T, ts.cam->bg[1], C1);
    a.out_rgb[2 * a.P + pix] = fmaf(T, ts.cam->bg[2], C2);
    a.out_T[pix] = T;
    a.out_last[pix] = last;
    if (CNT) {
      if (a.out_count) a.out_count[pix] = count;
      if (a.out_eval) a.out_eval[pix] = evals;
    }
  }
}

// CNT: also count evaluated and composited pairs per pixel (out_eval,
// out_count); the variant without them skips the counting instructions.
// QL: the tiles walk quarter lists (fwd_tile_q), whose staging holds more
// registers; six waves per SIMD measured fastest for it (the compiler's own
// choice, four, was slower than the wave lists); fewer where the enhanced
// opacity, the counters or 256-record batches would spill at six (8x8 tiles:
// their LDS already allows fewer).  The plain wave-list kernel of 16x16
// tiles fits 64 registers without spilling: eight waves per SIMD (1M
// forward blend 189 -> 177 us); its enhanced and counting variants would
// spill there.
template <int TW, int TH, int B, bool ENH, bool CNT, bool QL>
__global__ void __launch_bounds__(TW * TH)
    __attribute__((amdgpu_waves_per_eu(QL && TW * TH >= 128 ? (B > 128 || (ENH && CNT) ? 4 : (ENH || CNT ? 5 : 6))
                                                            : (!QL && !ENH && !CNT && TW * TH == 256 ? 8 : 1))))
    k_blend_fwd(BlendArgs a) {
  __shared__ Stage<TW, TH, B, ENH, QL ? TW * TH / 16 : TW * TH / 64> S;
  __shared__ uint32_t s_next;
  if (!a.work_counter) {
    if constexpr (TW == 16 && TH == 16) {
      if (blockIdx.x < 4u * (uint32_t)a.n_quad) {
        fwd_quad<B, ENH, CNT>(a, (int)a.tile_order[blockIdx.x >> 2], (int)(blockIdx.x & 3u), S);
        return;
      }
    }
    if constexpr (QL)
      fwd_tile_q<TW, TH, B, ENH, CNT>(a, launch_tile(a), S);
    else
      fwd_tile<TW, TH, B, ENH, CNT>(a, launch_tile(a), S);
    return;
  }
  for (int tile = next_tile(a, &s_next); tile >= 0; tile = next_tile(a, &s_next)) {
    if constexpr (QL)
      fwd_tile_q<TW, TH, B, ENH, CNT>(a, tile, S);
    else
      fwd_tile<TW, TH, B, ENH, CNT>(a, tile, S);
  }
}

template <int TW, int TH, int B, bool ENH>
struct BwdShared {
  static constexpr int NG = ENH ? 15 : 11;   // values per record: see the flush below
  Stage<TW, TH, B, ENH> S;
  static constexpr int SGW = B + 1;         // row stride: a record's slots in distinct banks
  float sg[NG][SGW];
  uint32_t smax;
};

// Writes a batch's per-record sums (LDS) to the 2D gradient planes.
template <int TW, int TH, int B, bool ENH>
__device__ __forceinline__ void flush_batch(const BlendArgs& a, int cnt, BwdShared<TW, TH, B, ENH>& X) {
  constexpr int NT = TW * TH;
  constexpr int NG = BwdShared<TW, TH, B, ENH>::NG;
  for (int k = threadIdx.x; k < cnt; k += NT) {
    float v[NG];
    bool any = false;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      v[q] = X.sg[q][k];
      any |= v[q] != 0.0f;
    }
    if (!any) continue;
    const uint32_t m = X.S.rid[k];
    float* p0 = reinterpret_cast<float*>(a.g0 + m);
    float* p1 = reinterpret_cast<float*>(a.g1 + m);
    float* p2 = reinterpret_cast<float*>(a.g2 + m);
    atomicAdd(p0 + 0, v[0]);
    atomicAdd(p0 + 1, v[1]);
    atomicAdd(p0 + 2, v[2]);
    atomicAdd(p0 + 3, v[3]);
    atomicAdd(p1 + 0, v[4]);
    atomicAdd(p1 + 1, v[5]);
    atomicAdd(p1 + 2, v[6]);
    atomicAdd(p1 + 3, v[7]);
    atomicAdd(p2 + 0, v[8]);
    atomicAdd(p2 + 1, v[9]);
    atomicAdd(p2 + 2, v[10]);
    if (ENH) {
      float* p3 = reinterpret_cast<float*>(a.g3 + m);
      atomicAdd(p3 + 0, v[11]);
      atomicAdd(p3 + 1, v[12]);
      atomicAdd(p3 + 2, v[13]);
      atomicAdd(p3 + 3, v[14]);
    }
  }
}

template <int TW, int TH, int B, bool ENH>
__device__ __forceinline__ void bwd_tile(const BlendArgs& a, int tile, BwdShared<TW, TH, B, ENH>& X) {
  constexpr int NT = TW * TH;
  constexpr int NG = BwdShared<TW, TH, B, ENH>::NG;
  auto& S = X.S;
  auto& sg = X.sg;
  uint32_t& smax = X.smax;
  TileSetup ts;
  if (!setup_tile<TW, TH>(a, tile, ts)) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const float fx = (float)ts.px + 0.5f, fy = (float)ts.py + 0.5f;
  uint2 rg = a.ranges[ts.tile];
  rg.y = min(rg.y, a.n_vals);
  rg.x = min(rg.x, rg.y);
  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  uint32_t last = 0;
  if (ts.inside) {
    const int64_t pix = ts.cam->pix_base + (int64_t)ts.py * ts.cam->width + ts.px;
    T = a.cT[pix];
    last = min(a.clast[pix], rg.y - rg.x);
    g0 = a.dL[pix];
    g1 = a.dL[a.P + pix];
    g2 = a.dL[2 * a.P + pix];
  }
  const float bgdot = ts.cam->bg[0] * g0 + ts.cam->bg[1] * g1 + ts.cam->bg[2] * g2;
  const float Tfinal = T;
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;   // colour behind, normalised
  if (t == 0) smax = 0;
  __syncthreads();
  if (last) atomicMax(&smax, last);
  __syncthreads();
  const int nmax = (int)smax;
  for (int end = nmax; end > 0; end -= B) {
    const int start = end > B ? end - B : 0;
    const int cnt = end - start;
    __syncthreads();
    stage_batch<TW, TH, B, ENH>(a, ts, rg.x + start, cnt, S);
    for (int k = t; k < NG * (B + 1); k += NT) (&sg[0][0])[k] = 0.0f;
    __syncthreads();
    const int nw = __builtin_amdgcn_readfirstlane(S.n[w]);   // wave-uniform
    for (int i = nw - 1; i >= 0; --i) {
      // j stays a per-lane value: with a wave-uniform LDS address the
      // compiler turns the atomics below into serial per-lane loops
      const uint32_t e = S.list[w][i];
      const int j = (int)(e & LIST_SLOT);
      const bool skew = ((uint32_t)__builtin_amdgcn_readfirstlane((int)e) & LIST_SKEW) != 0u;
      const float4 r0 = S.r0[j];
      const float4 r1 = S.r1[j];
      const float4 r2 = S.r2[j];
      const float dx = fx - r0.x, dy = fy - r0.y;
      const float l2 = pair_log2(r0.z, r0.w, r1.x, r1.w, dx, dy);
      const bool in = (uint32_t)(start + j) < last && l2 >= r2.w;
      // (guarded blocks rather than continue: the loop's control flow
      // then stays a plain counted loop in scalar code)
      if (wave_any(in)) {
        // from here on every lane computes; lanes without a contribution get
        // zero weights through selects (nested branches made the compiler
        // re-zero all gradient registers on every path)
        Pair2 p;
        pair_eval2(l2, r1.y, r1.z, dx, dy, skew, p);
        float at = p.at, o = 1.0f, eu = 0.0f, ee = 1.0f;
        float4 r3 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ENH) {
          r3 = S.r3[j];
          o = enh_opacity(r3.x, r3.y, r3.z, r3.w, dx, dy, eu, ee);
          at *= o;
        }
        const float alpha = fminf(a.alpha_max, at);
        const bool hit = in && alpha >= a.alpha_min;
        if (wave_any(hit)) {
          const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
          const float Tn = T * inv;                 // transmittance in front of this pair
          T = hit ? Tn : T;
          const float wgt = hit ? alpha * Tn : 0.0f;
          const bool unc = hit && at <= a.alpha_max;   // alpha not clamped: gradients reach it
          const float dLda = unc ? ((r2.x - S0) * g0 + (r2.y - S1) * g1 + (r2.z - S2) * g2) * Tn -
                                       Tfinal * inv * bgdot
                                 : 0.0f;
          const float ath = unc ? at : 0.0f;
          // common = dL/dalpha d o G'; (qa, qc) = Q delta and beta from the
          // staged base-2 constants
          const float common = unc ? dLda * o * p.dG : 0.0f;
          const float s2pi = SGS_SQRT_2_OVER_PI * p.ez;
          const float qa = -SGS_LN2 * fmaf(2.0f * r0.z, dx, r0.w * dy);
          const float qc = -SGS_LN2 * fmaf(r0.w, dx, 2.0f * r1.x * dy);
          float gv[NG];
          gv[0] = common * (qa * p.E - s2pi * (SGS_IKZ * r1.y));
          gv[1] = common * (qc * p.E - s2pi * (SGS_IKZ * r1.z));
          gv[2] = -0.5f * dx * dx * dLda * ath;
          gv[3] = -dx * dy * dLda * ath;
          gv[4] = -0.5f * dy * dy * dLda * ath;
          gv[5] = common * s2pi * dx;
          gv[6] = common * s2pi * dy;
          gv[7] = common * p.E * S.idv[j];
          gv[8] = wgt * g0;
          gv[9] = wgt * g1;
          gv[10] = wgt * g2;
          if constexpr (ENH) {
            const float base = unc ? p.at : 0.0f;        // rho G' (1 + erf z)
            const float dodw = (r3.x - r3.y) * SGS_INV_SQRT_2PI * ee;
            gv[0] -= dLda * base * dodw * r3.z;
            gv[1] -= dLda * base * dodw * r3.w;
            gv[11] = dLda * base * 0.5f * (1.0f + eu);
            gv[12] = dLda * base * 0.5f * (1.0f - eu);
            gv[13] = dLda * base * dodw * dx;
            gv[14] = dLda * base * dodw * dy;
          }
          S0 = hit ? fmaf(alpha, r2.x - S0, S0) : S0;
          S1 = hit ? fmaf(alpha, r2.y - S1, S1) : S1;
          S2 = hit ? fmaf(alpha, r2.z - S2, S2) : S2;
          // transposing sum over each 16-lane row (DPP): lane l of a row ends
          // with the row's sum of value l, then one LDS atomic per lane; the
          // VALU is this kernel's bound, the LDS pipe has room
          const float sv = row_transpose_sum<NG>(gv, lane);
          const int q = lane & 15;
          if (q < NG && sv != 0.0f) atomicAdd(&sg[q][j], sv);
        }
      }
    }
    __syncthreads();
    flush_batch<TW, TH, B, ENH>(a, cnt, X);
  }
}

// Backward of one 8x8 quarter of a 16x16 tile with four lanes per pixel
// (the counterpart of fwd_quad).  Per round the four lanes of a pixel take
// four consecutive records of the wave's list, walking backwards: each lane
// evaluates its record's alpha, the quad then runs the transmittance and
// colour-behind recursion over the four in list order (replicated, so T and
// S are those of bwd_tile bit for bit), and each lane computes its record's
// partial derivatives with the T and S in front of it.  Sums over the 16
// pixels that share a record take four shuffles.
template <int B, bool ENH>
__device__ __forceinline__ void bwd_quad(const BlendArgs& a, int tile, int quarter,
                                         BwdShared<16, 16, B, ENH>& X) {
  constexpr int NT = 256;
  constexpr int NG = BwdShared<16, 16, B, ENH>::NG;
  auto& S = X.S;
  auto& sg = X.sg;
  TileSetup ts;
  if (!setup_tile<16, 16>(a, tile, ts)) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, sub = lane & 3, pq = lane >> 2;
  ts.gx = ts.ox + (quarter & 1) * 8;
  ts.gy = ts.oy + (quarter >> 1) * 8;
  ts.px = ts.gx + (w & 1) * 4 + (pq & 3);
  ts.py = ts.gy + (w >> 1) * 4 + (pq >> 2);
  ts.inside = ts.px < ts.cam->width && ts.py < ts.cam->height;
  const float fx = (float)ts.px + 0.5f, fy = (float)ts.py + 0.5f;
  uint2 rg = a.ranges[ts.tile];
  rg.y = min(rg.y, a.n_vals);
  rg.x = min(rg.x, rg.y);
  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  uint32_t last = 0;
  if (ts.inside) {
    const int64_t pix = ts.cam->pix_base + (int64_t)ts.py * ts.cam->width + ts.px;
    T = a.cT[pix];
    last = min(a.clast[pix], rg.y - rg.x);
    g0 = a.dL[pix];
    g1 = a.dL[a.P + pix];
    g2 = a.dL[2 * a.P + pix];
  }
  const float bgdot = ts.cam->bg[0] * g0 + ts.cam->bg[1] * g1 + ts.cam->bg[2] * g2;
  const float Tfinal = T;
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
  if (t == 0) X.smax = 0;
  __syncthreads();
  if (last) atomicMax(&X.smax, last);
  __syncthreads();
  const int nmax = (int)X.smax;
  for (int end = nmax; end > 0; end -= B) {
    const int start = end > B ? end - B : 0;
    const int cnt = end - start;
    __syncthreads();
    stage_batch<16, 16, B, ENH, 4>(a, ts, rg.x + start, cnt, S);
    for (int k = t; k < NG * (B + 1); k += NT) (&sg[0][0])[k] = 0.0f;
    __syncthreads();
    const int nw = __builtin_amdgcn_readfirstlane(S.n[w]);   // wave-uniform
    for (int i = nw - 1; i >= 0; i -= 4) {
      const int k = i - sub;
      const bool has = k >= 0;
      const uint32_t e = has ? S.list[w][k] : 0u;
      const int j = (int)(e & LIST_SLOT);
      const float4 r0 = S.r0[j];
      const float4 r1 = S.r1[j];
      const float4 r2 = S.r2[j];
      const float dx = fx - r0.x, dy = fy - r0.y;
      const float l2 = pair_log2(r0.z, r0.w, r1.x, r1.w, dx, dy);
      const bool in = has && (uint32_t)(start + j) < last && l2 >= r2.w;
      Pair2 p;
      p.dG = p.E = p.ez = 1.0f;
      p.at = 0.0f;
      float at = 0.0f, o = 1.0f, eu = 0.0f, ee = 1.0f, alpha = 0.0f;
      float4 r3 = make_float4(0.f, 0.f, 0.f, 0.f);
      if (wave_any(in)) {
        pair_eval2(l2, r1.y, r1.z, dx, dy, (e & LIST_SKEW) != 0u, p);
        at = p.at;
        if (ENH) {
          r3 = S.r3[j];
          o = enh_opacity(r3.x, r3.y, r3.z, r3.w, dx, dy, eu, ee);
          at *= o;
        }
        alpha = fminf(a.alpha_max, at);
      }
      const bool hit = in && alpha >= a.alpha_min;
      if (wave_any(hit)) {   // (a guarded block rather than continue)
        // transmittance and colour-behind recursion, records in list order
        // (latest first), replicated on the quad
        const int hi = hit ? 1 : 0;
        const float cr = r2.x, cg = r2.y, cb = r2.z;
        float Tm = 0.0f, Sm0 = 0.0f, Sm1 = 0.0f, Sm2 = 0.0f;
  #define SGS_QUAD_BACK(Q)                                                     \
        if (quad_bcast<Q>(hi)) {                                               \
          const float al = quad_bcast<Q>(alpha);                               \
          T = T * __builtin_amdgcn_rcpf(1.0f - al);                            \
          if (sub == Q) {                                                      \
            Tm = T;                                                            \
            Sm0 = S0;                                                          \
            Sm1 = S1;                                                          \
            Sm2 = S2;                                                          \
          }                                                                    \
          S0 = fmaf(al, quad_bcast<Q>(cr) - S0, S0);                           \
          S1 = fmaf(al, quad_bcast<Q>(cg) - S1, S1);                           \
          S2 = fmaf(al, quad_bcast<Q>(cb) - S2, S2);                           \
        }
        SGS_QUAD_BACK(0)
        SGS_QUAD_BACK(1)
        SGS_QUAD_BACK(2)
        SGS_QUAD_BACK(3)
  #undef SGS_QUAD_BACK
        // every lane computes; lanes without a contribution get zero weights
        // through selects (no nested branches around the gradient registers)
        const float wgt = hit ? alpha * Tm : 0.0f;
        const bool unc = hit && at <= a.alpha_max;   // alpha not clamped: gradients reach it
        const float dLda = unc ? ((r2.x - Sm0) * g0 + (r2.y - Sm1) * g1 + (r2.z - Sm2) * g2) * Tm -
                                     Tfinal * __builtin_amdgcn_rcpf(1.0f - alpha) * bgdot
                               : 0.0f;
        const float ath = unc ? at : 0.0f;
        const float common = unc ? dLda * o * p.dG : 0.0f;
        const float s2pi = SGS_SQRT_2_OVER_PI * p.ez;
        const float qa = -SGS_LN2 * fmaf(2.0f * r0.z, dx, r0.w * dy);
        const float qc = -SGS_LN2 * fmaf(r0.w, dx, 2.0f * r1.x * dy);
        float gv[NG];
        gv[0] = common * (qa * p.E - s2pi * (SGS_IKZ * r1.y));
        gv[1] = common * (qc * p.E - s2pi * (SGS_IKZ * r1.z));
        gv[2] = -0.5f * dx * dx * dLda * ath;
        gv[3] = -dx * dy * dLda * ath;
        gv[4] = -0.5f * dy * dy * dLda * ath;
        gv[5] = common * s2pi * dx;
        gv[6] = common * s2pi * dy;
        gv[7] = common * p.E * S.idv[j];
        gv[8] = wgt * g0;
        gv[9] = wgt * g1;
        gv[10] = wgt * g2;
        if constexpr (ENH) {
          const float base = unc ? p.at : 0.0f;
          const float dodw = (r3.x - r3.y) * SGS_INV_SQRT_2PI * ee;
          gv[0] -= dLda * base * dodw * r3.z;
          gv[1] -= dLda * base * dodw * r3.w;
          gv[11] = dLda * base * 0.5f * (1.0f + eu);
          gv[12] = dLda * base * 0.5f * (1.0f - eu);
          gv[13] = dLda * base * dodw * dx;
          gv[14] = dLda * base * dodw * dy;
        }
        // sums over the 16 pixels of each sublane (lanes equal mod 4): within
        // a row by DPP row rotations by 4 and 8, across rows by shuffles;
        // lanes 0..3 hold sublanes 0..3
  #pragma unroll
        for (int q = 0; q < NG; ++q) {
          float v = gv[q];
          v += dpp_src<0x124>(v);   // row_ror:4
          v += dpp_src<0x128>(v);   // row_ror:8
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          if (lane < 4 && has && v != 0.0f) atomicAdd(&sg[q][j], v);
        }
      }
    }
    __syncthreads();
    flush_batch<16, 16, B, ENH>(a, cnt, X);
  }
}

template <int TW, int TH, int B, bool ENH>
__global__ void __launch_bounds__(TW * TH) k_blend_bwd(BlendArgs a) {
  __shared__ BwdShared<TW, TH, B, ENH> X;
  __shared__ uint32_t s_next;
  if (!a.work_counter) {
    if constexpr (TW == 16 && TH == 16) {
      if (blockIdx.x < 4u * (uint32_t)a.n_quad) {
        bwd_quad<B, ENH>(a, (int)a.tile_order[blockIdx.x >> 2], (int)(blockIdx.x & 3u), X);
        return;
      }
    }
    bwd_tile<TW, TH, B, ENH>(a, launch_tile(a), X);
    return;
  }
  for (int tile = next_tile(a, &s_next); tile >= 0; tile = next_tile(a, &s_next)) {
    bwd_tile<TW, TH, B, ENH>(a, tile, X);
    __syncthreads();
  }
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

// ------------------------------------------------------------------ launchers
// Workgroups that fit on the device at once (persistent launches).
template <typename F>
static unsigned resident_grid(F kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) return 0;
  return (unsigned)(cus * (per > 0 ? per : 1));
}

template <int TW, int TH, int B, bool ENH, bool QL>
static void launch_fwd_q(const BlendArgs& a, unsigned grid, hipStream_t s) {
  auto k = (a.out_count || a.out_eval) ? k_blend_fwd<TW, TH, B, ENH, true, QL>
                                       : k_blend_fwd<TW, TH, B, ENH, false, QL>;
  if (a.work_counter) {
    const unsigned g = resident_grid(k, TW * TH);
    grid = g ? std::min(g, grid) : grid;
    k_zero_u32<<<1, 1, 0, s>>>(a.work_counter);
  }
  k<<<grid, TW * TH, 0, s>>>(a);
}
template <int TW, int TH, int B, bool ENH>
static void launch_fwd_t(const BlendArgs& a, unsigned grid, hipStream_t s) {
  if (a.quarter_lists)
    launch_fwd_q<TW, TH, B, ENH, true>(a, grid, s);
  else
    launch_fwd_q<TW, TH, B, ENH, false>(a, grid, s);
}
template <int TW, int TH, int B, bool ENH>
static void launch_bwd_t(const BlendArgs& a, unsigned grid, hipStream_t s) {
  auto k = k_blend_bwd<TW, TH, B, ENH>;
  if (a.work_counter) {
    const unsigned g = resident_grid(k, TW * TH);
    grid = g ? std::min(g, grid) : grid;
    k_zero_u32<<<1, 1, 0, s>>>(a.work_counter);
  }
  k<<<grid, TW * TH, 0, s>>>(a);
}

template <bool BWD, int TW, int TH, bool ENH>
static sgs_status dispatch_b(const BlendArgs& a, int batch, unsigned grid, hipStream_t s) {
  switch (batch) {
    case 64: BWD ? launch_bwd_t<TW, TH, 64, ENH>(a, grid, s) : launch_fwd_t<TW, TH, 64, ENH>(a, grid, s); break;
    case 128: BWD ? launch_bwd_t<TW, TH, 128, ENH>(a, grid, s) : launch_fwd_t<TW, TH, 128, ENH>(a, grid, s); break;
    case 256: BWD ? launch_bwd_t<TW, TH, 256, ENH>(a, grid, s) : launch_fwd_t<TW, TH, 256, ENH>(a, grid, s); break;
    default: return SGS_EUNSUPPORTED;
  }
  SGS_LAUNCH_CHECK();
  return SGS_OK;
}

// blend_batch 0: 128 records per batch forward, 256 backward (measured best
// for each on the 300k and 1M workloads, except the backward at 300k)
template <bool BWD, bool ENH>
static sgs_status dispatch_tile(const BlendArgs& a, const sgs_options* opt, unsigned grid,
                                hipStream_t s) {
  const int bb = opt->blend_batch > 0 ? opt->blend_batch : (BWD ? 256 : 128);
  if (opt->tile_w == 16 && opt->tile_h == 16) return dispatch_b<BWD, 16, 16, ENH>(a, bb, grid, s);
  if (opt->tile_w == 16 && opt->tile_h == 8) return dispatch_b<BWD, 16, 8, ENH>(a, bb, grid, s);
  if (opt->tile_w == 8 && opt->tile_h == 8) return dispatch_b<BWD, 8, 8, ENH>(a, bb, grid, s);
  return SGS_EUNSUPPORTED;
}

static BlendArgs make_args(const sgs_geom* g, int64_t m, const uint32_t* vals, int64_t cap,
                           const uint32_t* ranges, const sgs_schedule* sched,
                           const sgs_camera* cams_dev, int32_t n_views, int64_t total_tiles,
                           const sgs_options* opt, int64_t P) {
  BlendArgs a = {};
  if (sched) {
    a.tile_order = sched->tile_order;
    a.work_counter = sched->work_counter;
  }
  a.rec = reinterpret_cast<const float4*>(g->rec);
  a.vals = vals;
  a.n_vals = (uint32_t)cap;
  a.ranges = reinterpret_cast<const uint2*>(ranges);
  a.cams = cams_dev;
  a.n_views = n_views;
  a.total_tiles = (int32_t)total_tiles;
  a.m = (uint32_t)m;
  a.alpha_min = opt->alpha_min;
  a.alpha_max = opt->alpha_max;
  a.t_min = opt->t_min;
  a.P = P;
  return a;
}

static unsigned blend_grid(int64_t total_tiles) { return (unsigned)((total_tiles + 7) / 8 * 8); }

// Split tiles (16x16 tiles with a tile order, no work counter): the first
// n_quad tiles of the order get four workgroups each, ahead of the others.
static void split_setup(BlendArgs& a, const sgs_options* opt, int64_t total_tiles, unsigned& grid) {
  if (a.tile_order && !a.work_counter && opt->tile_w == 16 && opt->tile_h == 16 && opt->split_tiles != 0) {
    const int64_t q = opt->split_tiles < 0 ? total_tiles / 128 : std::min<int64_t>(opt->split_tiles, total_tiles);
    a.n_quad = (int32_t)q;
    grid += 3u * (unsigned)q;
  }
}

sgs_status launch_blend_fwd(const sgs_geom* g, int64_t m, const uint32_t* vals, int64_t cap,
                            const uint32_t* ranges, const sgs_schedule* sched,
                            const sgs_camera* cams_dev, int32_t n_views,
                            int64_t total_tiles, int enhanced, const sgs_options* opt,
                            float* out_rgb, float* out_T, uint32_t* out_last,
                            uint32_t* out_count, uint32_t* out_eval, int64_t P, hipStream_t s) {
  BlendArgs a = make_args(g, m, vals, cap, ranges, sched, cams_dev, n_views, total_tiles, opt, P);
  a.out_rgb = out_rgb;
  a.out_T = out_T;
  a.out_last = out_last;
  a.out_count = out_count;
  a.out_eval = out_eval;
  unsigned grid = blend_grid(total_tiles);
  split_setup(a, opt, total_tiles, grid);
  // quarter lists where records are small: at most 8 instances of capacity
  // per record (1.65 for 300k Gaussians at 1280x720, where they shorten the
  // wave lists by 1.37x; about 65 for 1M at 1600x1064, where 1.04x does not
  // pay for their dearer steps)
  a.quarter_lists = opt->blend_lists == 4 || (opt->blend_lists == 0 && cap <= 8 * m);
  return enhanced ? dispatch_tile<false, true>(a, opt, grid, s)
                  : dispatch_tile<false, false>(a, opt, grid, s);
}

sgs_status launch_blend_bwd(const sgs_geom* g, int64_t m, const uint32_t* vals, int64_t cap,
                            const uint32_t* ranges, const sgs_schedule* sched,
                            const sgs_camera* cams_dev, int32_t n_views,
                            int64_t total_tiles, int enhanced, const sgs_options* opt,
                            const float* out_T, const uint32_t* out_last, const float* dL,
                            int64_t P, float* g2d, hipStream_t s) {
  BlendArgs a = make_args(g, m, vals, cap, ranges, sched, cams_dev, n_views, total_tiles, opt, P);
  a.cT = out_T;
  a.clast = out_last;
  a.dL = dL;
  float4* gr = reinterpret_cast<float4*>(g2d);
  a.g0 = gr;
  a.g1 = gr + m;
  a.g2 = gr + 2 * m;
  a.g3 = gr + 3 * m;
  unsigned grid = blend_grid(total_tiles);
  split_setup(a, opt, total_tiles, grid);
  return enhanced ? dispatch_tile<true, true>(a, opt, grid, s)
                  : dispatch_tile<true, false>(a, opt, grid, s);
}

}  // namespace sgs
