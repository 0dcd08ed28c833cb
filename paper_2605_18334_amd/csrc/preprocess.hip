// Per-(view, Gaussian) projection of 3D skew Gaussians and its backward.
//
// Forward (one thread per record m = v*N + i, 256-thread blocks, SoA reads):
//   Sigma = R S S^T R^T from quaternion and log-scale (Sec. "Preliminary of
//   3D Gaussian Splatting"), camera transform, affine (EWA) Jacobian J,
//   B = J W M (M = R S), Sigma' = B B^T, filter sI, conic Q = (Sigma'+sI)^-1,
//   compensation rho = sqrt(det Sigma'/det(Sigma'+sI)) (appendix "Forward
//   Pass"), 2D skew of the skew-normal marginal beta_2D = Q v / sqrt(1 +
//   kappa - v^T Q v), v = B M^T beta, kappa = |M^T beta|^2, SH colour, and the
//   opacity-aware screen extent -> tile rect and tile count.  The block sums
//   of tile counts are scanned by k_scan_blocks.
// Backward (one thread per Gaussian, loop over views): the chain rule from
//   the 2D record gradients to mean, log-scale, quaternion, skew, opacity
//   logits, enhanced-opacity direction and SH coefficients.
#include "sgs_dev.h"

namespace sgs {

struct PreArgs {
  sgs_params p;
  const sgs_camera* cams;
  sgs_options opt;
  float* rec;
  float* depth;
  uint32_t* rect;
  uint32_t* tiles;
  uint32_t* block_sums;
  uint32_t* rows;        // per record: tile rows with at least one tile (optional)
  int64_t n;
  int64_t m;
  int32_t nbx;
  int32_t enhanced;
};

// Everything the forward computes for one (view, Gaussian), kept for the
// backward, which recomputes it rather than storing it.
struct Proj {
  float s[3], q[4], qn, R[3][3], M[3][3];
  float tx, ty, tz, txr, tyr, limx, limy;
  bool clx, cly;
  float J00, J02, J11, J12, A[2][3], B[2][3];
  float s00, s01, s11, det2, detf, a, b, c, rho;
  float mux, muy, o1, o2;
  // skew map for beta (k = 0) and for beta + dir (k = 1)
  float u[2][3], vv[2][2], qv[2][2], rr[2];
  bool kclamp[2];
  float b2x, b2y, w2x, w2y;
  float dir[3], dist, raw[3], rgb[3];
  bool valid;
};

// One Gaussian's parameters, loaded together at the start of a thread so
// that their latencies overlap (the projection branches on the depth and on
// the footprint before it would otherwise reach the later loads).
template <int DEG>
struct Raw {
  static constexpr int K = (DEG + 1) * (DEG + 1);
  float mean[3], ls[3], q[4], op, op2, sk[3], od[3];
  float sh[K * 3];   // [k][channel]
};

template <int DEG>
__device__ __forceinline__ void load_raw(const sgs_params& p, int64_t i, int64_t n, Raw<DEG>& r) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.mean[k] = p.mean[k * n + i];
    r.ls[k] = p.log_scale[k * n + i];
    r.sk[k] = p.skew ? p.skew[k * n + i] : 0.0f;
    r.od[k] = p.opa_dir ? p.opa_dir[k * n + i] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) r.q[k] = p.quat[k * n + i];
  r.op = p.opa_logit[i];
  r.op2 = p.opa2_logit ? p.opa2_logit[i] : 0.0f;
#pragma unroll
  for (int k = 0; k < Raw<DEG>::K * 3; ++k) r.sh[k] = p.sh[(int64_t)k * n + i];
}

__device__ __forceinline__ void skew_map(const Proj& P, const float g[3], int k, Proj& Q) {
  float u0 = P.M[0][0] * g[0] + P.M[1][0] * g[1] + P.M[2][0] * g[2];
  float u1 = P.M[0][1] * g[0] + P.M[1][1] * g[1] + P.M[2][1] * g[2];
  float u2 = P.M[0][2] * g[0] + P.M[1][2] * g[1] + P.M[2][2] * g[2];
  float v0 = P.B[0][0] * u0 + P.B[0][1] * u1 + P.B[0][2] * u2;
  float v1 = P.B[1][0] * u0 + P.B[1][1] * u1 + P.B[1][2] * u2;
  float kappa = u0 * u0 + u1 * u1 + u2 * u2;
  float qv0 = P.a * v0 + P.b * v1;
  float qv1 = P.b * v0 + P.c * v1;
  float mq = v0 * qv0 + v1 * qv1;
  float km = kappa - mq;
  Q.kclamp[k] = !(km > 0.0f);
  float r = rsqrtf(1.0f + fmaxf(km, 0.0f));
  Q.u[k][0] = u0; Q.u[k][1] = u1; Q.u[k][2] = u2;
  Q.vv[k][0] = v0; Q.vv[k][1] = v1;
  Q.qv[k][0] = qv0; Q.qv[k][1] = qv1;
  Q.rr[k] = r;
}

template <int DEG>
__device__ __forceinline__ void project_fwd(const sgs_params& p, const Raw<DEG>& raw,
                                            const sgs_camera& cam, const sgs_options& opt,
                                            Proj& P) {
  const float mx = raw.mean[0], my = raw.mean[1], mz = raw.mean[2];
  const float* W = cam.w2c;
  P.tz = fmaf(W[8], mx, fmaf(W[9], my, fmaf(W[10], mz, W[11])));
  P.valid = (P.tz > cam.near_z) && isfinite(P.tz);
  if (!P.valid) return;
  P.tx = fmaf(W[0], mx, fmaf(W[1], my, fmaf(W[2], mz, W[3])));
  P.ty = fmaf(W[4], mx, fmaf(W[5], my, fmaf(W[6], mz, W[7])));
  // activations and M = R diag(s)
  for (int k = 0; k < 3; ++k) P.s[k] = __expf(raw.ls[k]);
  float qw = raw.q[0], qx = raw.q[1], qy = raw.q[2], qz = raw.q[3];
  P.qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float iq = 1.0f / P.qn;
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  P.q[0] = qw; P.q[1] = qx; P.q[2] = qy; P.q[3] = qz;
  P.R[0][0] = 1.f - 2.f * (qy * qy + qz * qz);
  P.R[0][1] = 2.f * (qx * qy - qw * qz);
  P.R[0][2] = 2.f * (qx * qz + qw * qy);
  P.R[1][0] = 2.f * (qx * qy + qw * qz);
  P.R[1][1] = 1.f - 2.f * (qx * qx + qz * qz);
  P.R[1][2] = 2.f * (qy * qz - qw * qx);
  P.R[2][0] = 2.f * (qx * qz - qw * qy);
  P.R[2][1] = 2.f * (qy * qz + qw * qx);
  P.R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) P.M[r][c] = P.R[r][c] * P.s[c];
  // affine approximation of the perspective map at t (EWA), with clamp
  const float itz = 1.0f / P.tz;
  P.txr = P.tx * itz;
  P.tyr = P.ty * itz;
  P.limx = opt.guard * (0.5f * (float)cam.width / cam.fx);
  P.limy = opt.guard * (0.5f * (float)cam.height / cam.fy);
  const float cxr = fminf(P.limx, fmaxf(-P.limx, P.txr));
  const float cyr = fminf(P.limy, fmaxf(-P.limy, P.tyr));
  P.clx = cxr != P.txr;
  P.cly = cyr != P.tyr;
  P.J00 = cam.fx * itz;
  P.J02 = -cam.fx * cxr * itz;
  P.J11 = cam.fy * itz;
  P.J12 = -cam.fy * cyr * itz;
  for (int c = 0; c < 3; ++c) {
    P.A[0][c] = fmaf(P.J00, W[c], P.J02 * W[8 + c]);
    P.A[1][c] = fmaf(P.J11, W[4 + c], P.J12 * W[8 + c]);
  }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      P.B[r][c] = P.A[r][0] * P.M[0][c] + P.A[r][1] * P.M[1][c] + P.A[r][2] * P.M[2][c];
  // Sigma' = B B^T; det by Cauchy-Binet (sum of squared 2x2 minors: no cancellation)
  P.s00 = P.B[0][0] * P.B[0][0] + P.B[0][1] * P.B[0][1] + P.B[0][2] * P.B[0][2];
  P.s01 = P.B[0][0] * P.B[1][0] + P.B[0][1] * P.B[1][1] + P.B[0][2] * P.B[1][2];
  P.s11 = P.B[1][0] * P.B[1][0] + P.B[1][1] * P.B[1][1] + P.B[1][2] * P.B[1][2];
  const float m01 = P.B[0][0] * P.B[1][1] - P.B[0][1] * P.B[1][0];
  const float m02 = P.B[0][0] * P.B[1][2] - P.B[0][2] * P.B[1][0];
  const float m12 = P.B[0][1] * P.B[1][2] - P.B[0][2] * P.B[1][1];
  P.det2 = m01 * m01 + m02 * m02 + m12 * m12;
  const float fs = opt.filter_s;
  P.detf = P.det2 + fs * (P.s00 + P.s11) + fs * fs;
  if (!(P.detf > 0.0f) || !isfinite(P.detf)) {
    P.valid = false;
    return;
  }
  const float idet = 1.0f / P.detf;
  P.a = (P.s11 + fs) * idet;
  P.b = -P.s01 * idet;
  P.c = (P.s00 + fs) * idet;
  P.rho = opt.compensate ? sqrtf(fmaxf(P.det2, 0.0f) * idet) : 1.0f;
  P.mux = fmaf(cam.fx, P.txr, cam.cx);
  P.muy = fmaf(cam.fy, P.tyr, cam.cy);
  P.o1 = 1.0f / (1.0f + __expf(-raw.op));
  P.o2 = p.opa2_logit ? 1.0f / (1.0f + __expf(-raw.op2)) : P.o1;
  // 2D skew: exact marginal of the skew-normal under B and the blur
  P.b2x = P.b2y = 0.0f;
  float beta[3] = {0.f, 0.f, 0.f};
  if (p.skew) {
    for (int k = 0; k < 3; ++k) beta[k] = raw.sk[k];
    skew_map(P, beta, 0, P);
    P.b2x = P.qv[0][0] * P.rr[0];
    P.b2y = P.qv[0][1] * P.rr[0];
  }
  P.w2x = P.w2y = 0.0f;
  if (p.opa2_logit) {
    float g[3];
    for (int k = 0; k < 3; ++k) g[k] = beta[k] + raw.od[k];
    skew_map(P, g, 1, P);
    P.w2x = P.qv[1][0] * P.rr[1];
    P.w2y = P.qv[1][1] * P.rr[1];
  }
  // view-dependent colour
  float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
  P.dist = sqrtf(dx * dx + dy * dy + dz * dz);
  const float id = 1.0f / P.dist;
  P.dir[0] = dx * id; P.dir[1] = dy * id; P.dir[2] = dz * id;
  float Y[16];
  sh_basis<DEG>(P.dir[0], P.dir[1], P.dir[2], Y);
  constexpr int K = (DEG + 1) * (DEG + 1);
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(Y[k], raw.sh[k * 3 + ch], acc);
    P.raw[ch] = acc;
    P.rgb[ch] = fmaxf(acc, 0.0f);
  }
  P.valid = isfinite(P.mux) && isfinite(P.muy) && isfinite(P.a) && isfinite(P.b) &&
            isfinite(P.c) && isfinite(P.b2x) && isfinite(P.b2y) && isfinite(P.w2x) &&
            isfinite(P.w2y);
}

// Tile counting runs per wave over (record, tile row) items: each lane
// projects its record and sets up its span, then the wave enumerates the
// rows of its 64 records 64 at a time (the owner's span is fetched with
// shuffles), so records with tall rects do not hold their wave back.
template <int DEG>
__global__ void __launch_bounds__(256) k_preprocess(PreArgs a) {
  __shared__ uint32_t s_pref[4][65];   // per wave: exclusive prefix of the records' rows
  __shared__ uint32_t s_cnt[256];
  __shared__ uint32_t s_ne[256];       // rows with at least one tile
  __shared__ float s_span[16][4][64];  // per field, wave and lane: the record's Span and tile rect
  __shared__ uint32_t s_mark[4][64];   // per wave: owner marks of the current row window
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  const int64_t m = (int64_t)v * a.n + i;
  const sgs_camera& cam = a.cams[v];
  Span sp;
  sp.ok = sp.cut = false;
  int tx0 = 0, tx1 = 0, ty0 = 0;
  uint32_t rows = 0, rx = 0, ry = 0;
  float tz = 0.0f;
  if (i < a.n) {
    Raw<DEG> raw;
    load_raw<DEG>(a.p, i, a.n, raw);
    Proj P;
    project_fwd<DEG>(a.p, raw, cam, a.opt, P);
    tz = P.tz;
    if (P.valid) {
      const bool has_skew = (P.b2x != 0.0f) || (P.b2y != 0.0f);
      const float dmax = P.rho * fmaxf(P.o1, P.o2);
      const float peak = dmax * (has_skew ? 2.0f : 1.0f);
      // alpha <= min(alpha_max, peak G') and G' <= 1: cull what never reaches alpha_min
      if (peak >= a.opt.alpha_min * (1.0f + 1e-4f)) {
        const float L = __logf(peak / a.opt.alpha_min);
        const float r2 = 2.0f * L * (1.0f + 1e-4f) + 1e-4f;      // ellipse delta^T Q delta <= r2
        const float ex = sqrtf(r2 * (P.s00 + a.opt.filter_s)) + 1e-2f;
        const float ey = sqrtf(r2 * (P.s11 + a.opt.filter_s)) + 1e-2f;
        // pixels whose centre (i + 0.5) lies in [mu - e, mu + e]
        float x0 = ceilf(P.mux - ex - 0.5f), x1 = floorf(P.mux + ex - 0.5f);
        float y0 = ceilf(P.muy - ey - 0.5f), y1 = floorf(P.muy + ey - 0.5f);
        if (isfinite(ex) && isfinite(ey)) {
          x0 = fmaxf(x0, 0.0f);
          y0 = fmaxf(y0, 0.0f);
          x1 = fminf(x1, (float)(cam.width - 1));
          y1 = fminf(y1, (float)(cam.height - 1));
          if (x0 <= x1 && y0 <= y1) {
            tx0 = (int)x0 / a.opt.tile_w;
            tx1 = (int)x1 / a.opt.tile_w + 1;
            ty0 = (int)y0 / a.opt.tile_h;
            const int ty1 = (int)y1 / a.opt.tile_h + 1;
            rx = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
            ry = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
            rows = (uint32_t)(ty1 - ty0);
            const float thr = -L - 1e-3f;   // power below thr => alpha < alpha_min
            // stored opacity factor: rho * alpha_1, or rho alone with enhanced
            // opacity (an upper bound of rho * o(delta), so the cut stays safe)
            const float d = a.enhanced ? P.rho : P.rho * P.o1;
            const float zc = has_skew ? skew_zcut(a.opt.alpha_min, d) : -1e30f;
            span_setup(P.mux, P.muy, P.a, P.b, P.c, thr, P.b2x, P.b2y, zc, sp);
            float4* rec = reinterpret_cast<float4*>(a.rec) + 4 * m;
            rec[0] = make_float4(P.mux, P.muy, P.a, P.b);
            rec[1] = make_float4(P.c, P.b2x, P.b2y, d);
            rec[2] = make_float4(P.rgb[0], P.rgb[1], P.rgb[2], thr);
            // slot 3: enhanced opacity, or else the rect (binning then
            // gathers this one line per record)
            rec[3] = a.enhanced ? make_float4(P.o1, P.o2, P.w2x, P.w2y)
                                : make_float4(__uint_as_float(rx), __uint_as_float(ry), 0.0f, 0.0f);
          }
        }
      }
    }
  }
  // tiles of each rect that the evaluation ellipse (cut by the skew
  // half-plane) reaches, row by row, per wave: the wave's (record, row)
  // items are spread over its lanes 64 at a time; each record's span and
  // rect sit in LDS, and an item finds its record by a max-scan of marks
  // (each record overlapping the window marks its first item there)
  const uint32_t incl = wave_incl_scan(rows);
  const uint32_t first = incl - rows;
  s_pref[w][lane] = first;
  if (lane == 63) s_pref[w][64] = incl;
  s_cnt[t] = 0;
  s_ne[t] = 0;
  {
    const float f[16] = {sp.mx, sp.my, sp.b, sp.det, sp.ia, sp.aR2, sp.ey, sp.ex,
                         sp.yx, sp.bx, sp.by, sp.need,
                         __uint_as_float((sp.ok ? 1u : 0u) | (sp.cut ? 2u : 0u)),
                         __int_as_float(tx0), __int_as_float(tx1), __int_as_float(ty0)};
#pragma unroll
    for (int k = 0; k < 16; ++k) s_span[k][w][lane] = f[k];
  }
  __syncthreads();
  const uint32_t R = s_pref[w][64];
  for (uint32_t base = 0; base < R; base += 64) {
    const uint32_t it = base + lane;
    s_mark[w][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    if (rows > 0 && first < base + 64 && incl > base)   // (positions of such records are distinct)
      s_mark[w][(first > base ? first : base) - base] = (uint32_t)lane + 1u;
    __builtin_amdgcn_wave_barrier();
    const int o = (int)wave_incl_max(s_mark[w][lane]) - 1;   // last record starting at or before it
    __builtin_amdgcn_wave_barrier();
    if (it < R) {
      float g[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) g[k] = s_span[k][w][o];   // (lanes read distinct banks)
      const float4 q0 = make_float4(g[0], g[1], g[2], g[3]), q1 = make_float4(g[4], g[5], g[6], g[7]);
      const float4 q2 = make_float4(g[8], g[9], g[10], g[11]), q3 = make_float4(g[12], g[13], g[14], g[15]);
      Span so;
      so.mx = q0.x; so.my = q0.y; so.b = q0.z; so.det = q0.w;
      so.ia = q1.x; so.aR2 = q1.y; so.ey = q1.z; so.ex = q1.w;
      so.yx = q2.x; so.bx = q2.y; so.by = q2.z; so.need = q2.w;
      so.ok = (__float_as_uint(q3.x) & 1u) != 0u;
      so.cut = (__float_as_uint(q3.x) & 2u) != 0u;
      int c0, c1;
      span_row(so, __float_as_int(q3.w) + (int)(it - s_pref[w][o]), a.opt.tile_w, a.opt.tile_h,
               __float_as_int(q3.y), __float_as_int(q3.z), c0, c1);
      if (c1 > c0) {
        atomicAdd(&s_cnt[w * 64 + o], (uint32_t)(c1 - c0));
        atomicAdd(&s_ne[w * 64 + o], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t ntiles = s_cnt[t];
  if (i < a.n) {
    // records without tiles get all-ones bits: they sort after every finite depth
    a.depth[m] = ntiles ? tz : __uint_as_float(0xffffffffu);
    a.tiles[m] = ntiles;
    if (a.rows) a.rows[m] = s_ne[t];
    reinterpret_cast<uint2*>(a.rect)[m] = make_uint2(rx, ry);
  }
  // block sum of tile counts (for the instance offsets)
  uint32_t s = ntiles;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ uint32_t ws[4];
  if (lane == 0) ws[w] = s;
  __syncthreads();
  if (t == 0) a.block_sums[(int64_t)v * a.nbx + blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of nb block sums into out[0..nb], out[nb] = total.  One
// block of 1024 threads, 8 consecutive entries per thread per round.  Sums
// are kept in 64 bits; an offset past 2^32 - 1 is written as 0xffffffff (the
// caller sees a saturated total and rejects the frame).
__global__ void __launch_bounds__(1024) k_scan_blocks(const uint32_t* __restrict__ in,
                                                      uint32_t* __restrict__ out, int64_t nb) {
  __shared__ uint64_t wsum[16];
  __shared__ uint64_t carry_s;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) carry_s = 0;
  __syncthreads();
  auto sat = [](uint64_t x) { return x > 0xffffffffull ? 0xffffffffu : (uint32_t)x; };
  for (int64_t base = 0; base < nb; base += 8192) {
    uint64_t v[8];
    uint64_t loc = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t idx = base + (int64_t)t * 8 + k;
      const uint64_t x = idx < nb ? (uint64_t)in[idx] : 0ull;
      v[k] = loc;
      loc += x;
    }
    uint64_t inc = loc;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
      const uint64_t ws = lane < 16 ? wsum[lane] : 0ull;
      uint64_t wi = ws;
      for (int off = 1; off < 16; off <<= 1) {
        const uint64_t y = __shfl_up(wi, off);
        if (lane >= off) wi += y;
      }
      if (lane < 16) wsum[lane] = wi - ws;   // exclusive wave offsets
    }
    __syncthreads();
    const uint64_t pre = carry_s + wsum[w] + inc - loc;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t idx = base + (int64_t)t * 8 + k;
      if (idx < nb) out[idx] = sat(pre + v[k]);
    }
    __syncthreads();
    if (t == 1023) carry_s = pre + loc;
    __syncthreads();
  }
  if (t == 0) out[nb] = sat(carry_s);
}

// ------------------------------------------------------------------ backward
struct PreBwdArgs {
  sgs_params p;
  const sgs_camera* cams;
  sgs_options opt;
  const uint32_t* tiles;
  const float* g2d;   // [R][M][4]
  sgs_params_grad g;
  int64_t n;
  int64_t m;
  int32_t n_views;
  int32_t enhanced;
};

// Backward of the skew map k for upstream gradient (gx, gy) of the 2D skew.
// Accumulates into gvec (the 3D input vector), gM, gB and the symmetric
// full-matrix gradient GQ of the conic.
__device__ __forceinline__ void skew_map_bwd(const Proj& P, int k, const float g3[3], float gx,
                                             float gy, float gvec[3], float gM[3][3],
                                             float gB[2][3], float GQ[2][2]) {
  const float r = P.rr[k];
  const float gqv0 = gx * r, gqv1 = gy * r;
  const float grr = gx * P.qv[k][0] + gy * P.qv[k][1];
  float gk = 0.0f, gmq = 0.0f;
  if (!P.kclamp[k]) {
    const float r3 = r * r * r;
    gk = -0.5f * r3 * grr;
    gmq = 0.5f * r3 * grr;
  }
  const float v0 = P.vv[k][0], v1 = P.vv[k][1];
  // qv = Q v, mq = v . qv
  const float gv0 = P.a * gqv0 + P.b * gqv1 + 2.0f * P.qv[k][0] * gmq;
  const float gv1 = P.b * gqv0 + P.c * gqv1 + 2.0f * P.qv[k][1] * gmq;
  GQ[0][0] += gqv0 * v0 + gmq * v0 * v0;
  GQ[1][1] += gqv1 * v1 + gmq * v1 * v1;
  const float off = 0.5f * (gqv0 * v1 + gqv1 * v0) + gmq * v0 * v1;
  GQ[0][1] += off;
  GQ[1][0] += off;
  // kappa = |u|^2, v = B u, u = M^T g
  float gu[3];
  for (int j = 0; j < 3; ++j) {
    gu[j] = 2.0f * P.u[k][j] * gk + P.B[0][j] * gv0 + P.B[1][j] * gv1;
    gB[0][j] += gv0 * P.u[k][j];
    gB[1][j] += gv1 * P.u[k][j];
  }
  for (int r2 = 0; r2 < 3; ++r2) {
    gvec[r2] += P.M[r2][0] * gu[0] + P.M[r2][1] * gu[1] + P.M[r2][2] * gu[2];
    for (int j = 0; j < 3; ++j) gM[r2][j] += g3[r2] * gu[j];
  }
}

template <int DEG>
__global__ void __launch_bounds__(256) k_preprocess_bwd(PreBwdArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n, M = a.m;
  constexpr int K = (DEG + 1) * (DEG + 1);
  float gmean[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0};
  float gbeta[3] = {0, 0, 0}, gdirv3[3] = {0, 0, 0};
  float gl1 = 0.0f, gl2 = 0.0f;
  float st_uv = 0.0f, st_z = 0.0f;   // densification statistics over the views
  uint32_t st_n = 0;
  const float4* g2 = reinterpret_cast<const float4*>(a.g2d);
  Raw<DEG> raw;
  load_raw<DEG>(a.p, i, n, raw);
  for (int v = 0; v < a.n_views; ++v) {
    const int64_t m = (int64_t)v * n + i;
    if (a.tiles[m] == 0) continue;
    const sgs_camera& cam = a.cams[v];
    Proj P;
    project_fwd<DEG>(a.p, raw, cam, a.opt, P);
    if (!P.valid) continue;
    const float4 G0 = g2[m], G1 = g2[M + m], G2 = g2[2 * M + m];
    const float4 G3 = a.enhanced ? g2[3 * M + m] : make_float4(0.f, 0.f, 0.f, 0.f);
    // opacity: d = rho * alpha_1 (or rho alone with enhanced opacity)
    float grho, go1, go2 = 0.0f;
    if (a.enhanced) {
      grho = G1.w;
      go1 = G3.x;
      go2 = G3.y;
    } else {
      grho = G1.w * P.o1;
      go1 = G1.w * P.rho;
    }
    gl1 += go1 * P.o1 * (1.0f - P.o1);
    if (a.p.opa2_logit) gl2 += go2 * P.o2 * (1.0f - P.o2);
    // conic gradient from the blend: b is the off-diagonal, counted once
    float GQ[2][2] = {{G0.z, 0.5f * G0.w}, {0.5f * G0.w, G1.x}};
    float gM[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    float gB[2][3] = {{0, 0, 0}, {0, 0, 0}};
    float beta[3] = {0, 0, 0};
    if (a.p.skew) {
      for (int k = 0; k < 3; ++k) beta[k] = a.p.skew[k * n + i];
      skew_map_bwd(P, 0, beta, G1.y, G1.z, gbeta, gM, gB, GQ);
    }
    if (a.p.opa2_logit) {
      float g3[3], gv[3] = {0, 0, 0};
      for (int k = 0; k < 3; ++k) g3[k] = beta[k] + (a.p.opa_dir ? a.p.opa_dir[k * n + i] : 0.f);
      skew_map_bwd(P, 1, g3, G3.z, G3.w, gv, gM, gB, GQ);
      for (int k = 0; k < 3; ++k) {
        if (a.p.skew) gbeta[k] += gv[k];
        gdirv3[k] += gv[k];
      }
    }
    // Q = Sigma_f^-1: G_Sigma_f = -Q GQ Q
    const float Qm[2][2] = {{P.a, P.b}, {P.b, P.c}};
    float T[2][2], GS[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) T[r][c] = Qm[r][0] * GQ[0][c] + Qm[r][1] * GQ[1][c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) GS[r][c] = -(T[r][0] * Qm[0][c] + T[r][1] * Qm[1][c]);
    // rho = sqrt(det Sigma' / det Sigma_f): d rho = rho/2 (adj(S')/det' - Q) : dS'
    if (a.opt.compensate && P.det2 > 0.0f && grho != 0.0f) {
      const float h = 0.5f * P.rho * grho;
      const float id2 = 1.0f / P.det2;
      GS[0][0] += h * (P.s11 * id2 - P.a);
      GS[1][1] += h * (P.s00 * id2 - P.c);
      GS[0][1] += h * (-P.s01 * id2 - P.b);
      GS[1][0] += h * (-P.s01 * id2 - P.b);
    }
    // Sigma' = B B^T
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        gB[r][c] += (GS[r][0] + GS[0][r]) * P.B[0][c] + (GS[r][1] + GS[1][r]) * P.B[1][c];
    // B = A M
    float gA[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        gA[r][c] = gB[r][0] * P.M[c][0] + gB[r][1] * P.M[c][1] + gB[r][2] * P.M[c][2];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) gM[r][c] += P.A[0][r] * gB[0][c] + P.A[1][r] * gB[1][c];
    // A = J W
    const float* W = cam.w2c;
    const float gJ00 = gA[0][0] * W[0] + gA[0][1] * W[1] + gA[0][2] * W[2];
    const float gJ02 = gA[0][0] * W[8] + gA[0][1] * W[9] + gA[0][2] * W[10];
    const float gJ11 = gA[1][0] * W[4] + gA[1][1] * W[5] + gA[1][2] * W[6];
    const float gJ12 = gA[1][0] * W[8] + gA[1][1] * W[9] + gA[1][2] * W[10];
    const float itz = 1.0f / P.tz, itz2 = itz * itz;
    float gtx = 0.0f, gty = 0.0f, gtz = -(gJ00 * cam.fx + gJ11 * cam.fy) * itz2;
    if (!P.clx) {
      gtx += -gJ02 * cam.fx * itz2;
      gtz += gJ02 * 2.0f * cam.fx * P.tx * itz2 * itz;
    } else {
      gtz += gJ02 * cam.fx * fminf(P.limx, fmaxf(-P.limx, P.txr)) * itz2;
    }
    if (!P.cly) {
      gty += -gJ12 * cam.fy * itz2;
      gtz += gJ12 * 2.0f * cam.fy * P.ty * itz2 * itz;
    } else {
      gtz += gJ12 * cam.fy * fminf(P.limy, fmaxf(-P.limy, P.tyr)) * itz2;
    }
    // 2D mean
    gtx += G0.x * cam.fx * itz;
    gty += G0.y * cam.fy * itz;
    gtz -= (G0.x * cam.fx * P.tx + G0.y * cam.fy * P.ty) * itz2;
    float gmv[3];   // this view's gradient w.r.t. the mean
    for (int k = 0; k < 3; ++k) gmv[k] = W[k] * gtx + W[4 + k] * gty + W[8 + k] * gtz;
    // M = R diag(s)
    float gR[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) gR[r][c] = gM[r][c] * P.s[c];
    for (int c = 0; c < 3; ++c)
      gls[c] += (gM[0][c] * P.R[0][c] + gM[1][c] * P.R[1][c] + gM[2][c] * P.R[2][c]) * P.s[c];
    const float w = P.q[0], x = P.q[1], y = P.q[2], z = P.q[3];
    float gqn[4];
    gqn[0] = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    gqn[1] = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.f * x * gR[1][1] - w * gR[1][2] +
                    z * gR[2][0] + w * gR[2][1] - 2.f * x * gR[2][2]);
    gqn[2] = 2.f * (-2.f * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                    w * gR[2][0] + z * gR[2][1] - 2.f * y * gR[2][2]);
    gqn[3] = 2.f * (-2.f * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.f * z * gR[1][1] +
                    y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const float dotq = w * gqn[0] + x * gqn[1] + y * gqn[2] + z * gqn[3];
    const float iqn = 1.0f / P.qn;
    for (int k = 0; k < 4; ++k) gq[k] += (gqn[k] - P.q[k] * dotq) * iqn;
    // colour: rgb = max(0, sum_k Y_k sh_k + 0.5)
    const float gc[3] = {P.raw[0] > 0.f ? G2.x : 0.f, P.raw[1] > 0.f ? G2.y : 0.f,
                         P.raw[2] > 0.f ? G2.z : 0.f};
    if (gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f) {
      float Y[16], wk[16];
      sh_basis<DEG>(P.dir[0], P.dir[1], P.dir[2], Y);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float acc = 0.0f;
        for (int ch = 0; ch < 3; ++ch) {
          const int64_t idx = ((int64_t)k * 3 + ch) * n + i;
          acc += gc[ch] * a.p.sh[idx];
          if (a.g.sh) a.g.sh[idx] += gc[ch] * Y[k];
        }
        wk[k] = acc;
      }
      if (DEG > 0) {
        float gdx, gdy, gdz;
        sh_basis_grad<DEG>(P.dir[0], P.dir[1], P.dir[2], wk, gdx, gdy, gdz);
        const float dd = gdx * P.dir[0] + gdy * P.dir[1] + gdz * P.dir[2];
        const float idist = 1.0f / P.dist;
        gmv[0] += (gdx - P.dir[0] * dd) * idist;
        gmv[1] += (gdy - P.dir[1] * dd) * idist;
        gmv[2] += (gdz - P.dir[2] * dd) * idist;
      }
    }
    for (int k = 0; k < 3; ++k) gmean[k] += gmv[k];
    // densification statistics (Sec. "Depth-Aware Densification Strategy"):
    // screen-space gradient norm in NDC units (pixels scale by W/2, H/2) and
    // the derivative along this view's depth axis (third row of w2c)
    const float gu = G0.x * (0.5f * (float)cam.width), gv = G0.y * (0.5f * (float)cam.height);
    st_uv += sqrtf(gu * gu + gv * gv);
    st_z = fmaxf(st_z, fabsf(W[8] * gmv[0] + W[9] * gmv[1] + W[10] * gmv[2]));
    ++st_n;
  }
  if (a.g.densify_uv) a.g.densify_uv[i] += st_uv;
  if (a.g.densify_z) a.g.densify_z[i] = fmaxf(a.g.densify_z[i], st_z);
  if (a.g.densify_count) a.g.densify_count[i] += st_n;
  for (int k = 0; k < 3; ++k) {
    if (a.g.mean) a.g.mean[k * n + i] += gmean[k];
    if (a.g.log_scale) a.g.log_scale[k * n + i] += gls[k];
    if (a.g.skew && a.p.skew) a.g.skew[k * n + i] += gbeta[k];
    if (a.g.opa_dir && a.p.opa_dir) a.g.opa_dir[k * n + i] += gdirv3[k];
  }
  for (int k = 0; k < 4; ++k)
    if (a.g.quat) a.g.quat[k * n + i] += gq[k];
  if (a.g.opa_logit) a.g.opa_logit[i] += gl1;
  if (a.g.opa2_logit && a.p.opa2_logit) a.g.opa2_logit[i] += gl2;
}

// ------------------------------------------------------------------ launchers
sgs_status launch_preprocess(const sgs_params* p, const sgs_camera* cams_dev, int32_t n_views,
                             const sgs_options* opt, const sgs_geom* g, hipStream_t s) {
  PreArgs a;
  a.p = *p;
  a.cams = cams_dev;
  a.opt = *opt;
  a.rec = g->rec;
  a.depth = g->depth;
  a.rect = g->rect;
  a.tiles = g->tiles;
  a.rows = g->rows;
  a.n = p->n;
  a.m = p->n * n_views;
  a.nbx = (int32_t)((p->n + 255) / 256);
  a.enhanced = p->opa2_logit != nullptr;
  const int64_t nb = (int64_t)a.nbx * n_views;
  // block sums live in the upper part of block_off; the scan writes below
  // them (out[k] only after in[k] of the same round was read by its thread)
  a.block_sums = g->block_off;
  if (nb > 0) {
    dim3 grid(a.nbx, n_views);
    switch (p->sh_degree) {
      case 0: k_preprocess<0><<<grid, 256, 0, s>>>(a); break;
      case 1: k_preprocess<1><<<grid, 256, 0, s>>>(a); break;
      case 2: k_preprocess<2><<<grid, 256, 0, s>>>(a); break;
      default: k_preprocess<3><<<grid, 256, 0, s>>>(a); break;
    }
    SGS_LAUNCH_CHECK();
  }
  k_scan_blocks<<<1, 1024, 0, s>>>(g->block_off, g->block_off, nb);
  SGS_LAUNCH_CHECK();
  return SGS_OK;
}

sgs_status launch_preprocess_bwd(const sgs_params* p, const sgs_camera* cams_dev,
                                 int32_t n_views, const sgs_options* opt, const sgs_geom* g,
                                 const float* g2d, const sgs_params_grad* grad, hipStream_t s) {
  PreBwdArgs a;
  a.p = *p;
  a.cams = cams_dev;
  a.opt = *opt;
  a.tiles = g->tiles;
  a.g2d = g2d;
  a.g = *grad;
  a.n = p->n;
  a.m = p->n * n_views;
  a.n_views = n_views;
  a.enhanced = p->opa2_logit != nullptr;
  if (p->n == 0) return SGS_OK;
  const unsigned nb = (unsigned)((p->n + 255) / 256);
  switch (p->sh_degree) {
    case 0: k_preprocess_bwd<0><<<nb, 256, 0, s>>>(a); break;
    case 1: k_preprocess_bwd<1><<<nb, 256, 0, s>>>(a); break;
    case 2: k_preprocess_bwd<2><<<nb, 256, 0, s>>>(a); break;
    default: k_preprocess_bwd<3><<<nb, 256, 0, s>>>(a); break;
  }
  SGS_LAUNCH_CHECK();
  return SGS_OK;
}

}  // namespace sgs
