// Device-side helpers shared by the HIP kernels of the skew-Gaussian
// rasterizer (gfx950, wave64).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgs.h"

#define SGS_INV_SQRT2 0.70710678118654752f
#define SGS_SQRT_2_OVER_PI 0.79788456080286536f   // sqrt(2/pi)
#define SGS_INV_SQRT_2PI 0.39894228040143268f      // 1/sqrt(2 pi)
#define SGS_L2E 1.44269504088896341f                // log2(e)
#define SGS_LN2 0.69314718055994531f                // ln(2) = 1/log2(e)
#define SGS_KA (-0.72134752044448170f)              // -log2(e)/2
#define SGS_KZ 0.84932180028801904f                 // sqrt(log2(e)/2)
#define SGS_IKZ 1.17741002251547466f                // 1/SGS_KZ

namespace sgs {

constexpr int kWave = 64;

// Checks the launch that was just enqueued.
#define SGS_LAUNCH_CHECK()                                   \
  do {                                                       \
    hipError_t e__ = hipGetLastError();                      \
    if (e__ != hipSuccess) return SGS_EHIP;                  \
  } while (0)

__device__ __forceinline__ float4 ld4(const float* p, int64_t i) {
  return reinterpret_cast<const float4*>(p)[i];
}

// ---------------------------------------------------------------- the pair
// alpha~ of one (pixel, record) pair, Alg. 1: G' = exp(-(a dx^2 + c dy^2)/2
// - b dx dy), z = (beta_x dx + beta_y dy)/sqrt 2, alpha~ = d G' (1 + erf z).
// Written with explicit fma so that the forward and the backward kernels
// evaluate bit-identical values (their decisions must agree).

// 1 + erf(z) = erfc(-z) with erfc(x) ~ t P(t) exp(-x^2), t = 1/(1 + p x),
// x >= 0 (Abramowitz & Stegun 1964, formula 7.1.26, |error| <= 1.5e-7), and
// erfc(-x) = 2 - erfc(x).  Also returns exp(-z^2), which the backward needs.
__device__ __forceinline__ float one_plus_erf(float z, float& ez) {
  const float x = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));   // v_rcp_f32 (1 ulp)
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  ez = __expf(-x * x);
  const float q = (poly * t) * ez;      // erfc(|z|)
  return z < 0.0f ? q : 2.0f - q;
}

// The kernels evaluate it in base 2, with per-record constants staged once
// per batch: log2(d G') = A dx^2 + B dx dy + C dy^2 + D with
// A = -(log2 e)/2 a, B = -(log2 e) b, C = -(log2 e)/2 c, D = log2 d, and the
// skew argument scaled by sqrt(log2 e): zs = bxs dx + bys dy = z sqrt(log2 e)
// with (bxs, bys) = sqrt(log2(e)/2) (beta_x, beta_y), so exp(-z^2) = 2^-zs^2.
// The skip test log2(d G') >= log2(e) log_thr + D is the exponent test of the
// natural form.  Forward and backward evaluate these same expressions.
struct Pair2 {
  float dG;     // d G'
  float E;      // 1 + erf(z)
  float ez;     // exp(-z^2) (1 when z = 0)
  float at;     // d G' (1 + erf z) (without the enhanced-opacity factor)
};

__device__ __forceinline__ float pair_log2(float A, float B, float C, float D, float dx, float dy) {
  return fmaf(fmaf(A, dx, B * dy), dx, fmaf(C * dy, dy, D));
}

// one_plus_erf of z = zs / sqrt(log2 e): t = 1/(1 + p x) with p x =
// (p / sqrt(log2 e)) |zs|, and exp(-x^2) = 2^(-zs^2).
__device__ __forceinline__ float one_plus_erf_s(float zs, float& ez) {
  const float x = fabsf(zs);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.27273747324943543f, x, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  ez = __builtin_amdgcn_exp2f(-(zs * zs));
  const float q = (poly * t) * ez;      // erfc(|z|)
  return zs < 0.0f ? q : 2.0f - q;
}

__device__ __forceinline__ void pair_eval2(float l2, float bxs, float bys, float dx, float dy,
                                           bool skew, Pair2& p) {
  p.dG = __builtin_amdgcn_exp2f(l2);
  if (skew) {
    p.E = one_plus_erf_s(fmaf(bxs, dx, bys * dy), p.ez);
  } else {
    p.E = 1.0f;
    p.ez = 1.0f;
  }
  p.at = p.dG * p.E;
}

// Enhanced opacity factor o(delta) = ((o1+o2) + (o1-o2) erf(w.delta/sqrt2))/2
// (Sec. "3D Skew Gaussian Rasterization and Splatting").
// Returns o(delta); erfu = erf(u), eu = exp(-u^2), u = w.delta/sqrt 2.
__device__ __forceinline__ float enh_opacity(float o1, float o2, float wx, float wy, float dx,
                                             float dy, float& erfu, float& eu) {
  const float u = fmaf(wx, dx, wy * dy) * SGS_INV_SQRT2;
  erfu = one_plus_erf(u, eu) - 1.0f;
  return 0.5f * fmaf(o1 - o2, erfu, o1 + o2);
}

// ---------------------------------------------------------------- tiles
// Skew cut: pairs whose z = beta.delta/sqrt2 is below the returned value have
// alpha <= d (1 + erf z) < alpha_min (G' <= 1), d the record's largest
// opacity factor.  1e-3 below the exact root of 1 + erf(z0) = alpha_min/d;
// since d <= 1, z0 >= -2.04 and the slope of 1 + erf there keeps that margin
// far above the float32 error of the evaluated alpha.  -1e30: no cut.
__device__ __forceinline__ float skew_zcut(float alpha_min, float d) {
  const float t = alpha_min / d - 1.0f;
  if (!(t > -1.0f)) return -1e30f;
  if (t >= 1.0f) return 1e30f;
  return erfinvf(t) - 1e-3f;
}

// Largest beta.delta over pixel centres of the box with centre (cx, cy) and
// half extents (hx, hy), delta = centre - mean.
__device__ __forceinline__ float skew_box_max(float bx, float by, float cx, float cy, float mx,
                                              float my, float hx, float hy) {
#pragma clang fp contract(off)
  return bx * (cx - mx) + by * (cy - my) + fabsf(bx) * hx + fabsf(by) * hy;
}

// Per-record extent of the pairs that can reach alpha_min, tile row by tile
// row.  Columns [c0, c1) of tile row `row` are those whose pixel centres
// (i + 0.5) the ellipse {delta : a dx^2 + 2 b dx dy + c dy^2 <= R2} around
// (mx, my), R2 = -2 log_thr (outside it every pair is skipped), reaches,
// widened by a small margin, clipped to the record's rect [x0, x1) and cut
// by the skew half-plane beta.delta >= sqrt2 zcut (linear in the column, so
// the kept tiles stay one interval).  span_setup does the per-record work
// once; span_row is cheap.  Counting (preprocess) and enumeration (duplicate,
// expand) call this same contraction-free code on the same stored record
// values, so they agree exactly.
struct Span {
  float mx, my, b, det, ia, aR2;
  float ey, ex, yx;
  float bx, by, need;    // skew cut (cut == false: none)
  bool ok, cut;
};

__device__ __forceinline__ void span_setup(float mx, float my, float a, float b, float c,
                                           float log_thr, float bx, float by, float zcut,
                                           Span& s) {
#pragma clang fp contract(off)
  s.mx = mx;
  s.my = my;
  s.b = b;
  const float R2 = -2.0f * log_thr * 1.002f + 1e-3f;
  s.det = a * c - b * b;
  s.ok = (s.det > 0.0f) && (R2 > 0.0f) && (a > 0.0f) && (c > 0.0f);
  s.ia = 1.0f / a;
  s.aR2 = a * R2;
  s.ey = sqrtf(R2 * a / s.det);
  s.ex = sqrtf(R2 * c / s.det);
  s.yx = -b * sqrtf(R2) / sqrtf(c * s.det);   // dy where x is largest on the ellipse
  s.bx = bx;
  s.by = by;
  s.need = zcut * 1.41421356f;                // beta.delta >= need
  s.cut = zcut > -1e29f && (bx != 0.0f || by != 0.0f);
}

__device__ __forceinline__ void span_row(const Span& s, int row, int tw, int th, int x0, int x1,
                                         int& c0, int& c1) {
#pragma clang fp contract(off)
  c0 = x0;
  c1 = x0;
  if (!s.ok) {
    c1 = x1;                                   // degenerate: keep the whole rect row
    return;
  }
  float u0 = ((float)(row * th) + 0.5f - 0.01f) - s.my;
  float u1 = ((float)(row * th + th) - 0.5f + 0.01f) - s.my;
  u0 = fmaxf(u0, -s.ey);
  u1 = fminf(u1, s.ey);
  if (!(u0 <= u1)) return;
  // (hardware square root and reciprocal, within an ulp or two: far inside
  // the widening margins below; every caller runs this same code)
  const float r0 = __builtin_amdgcn_sqrtf(fmaxf(s.aR2 - s.det * u0 * u0, 0.0f));
  const float r1 = __builtin_amdgcn_sqrtf(fmaxf(s.aR2 - s.det * u1 * u1, 0.0f));
  float xr = fmaxf((-s.b * u0 + r0) * s.ia, (-s.b * u1 + r1) * s.ia);
  float xl = fminf((-s.b * u0 - r0) * s.ia, (-s.b * u1 - r1) * s.ia);
  if (s.yx >= u0 && s.yx <= u1) xr = s.ex;
  if (-s.yx >= u0 && -s.yx <= u1) xl = -s.ex;
  // widen outwards on both sides: 0.1% of the offset plus 0.01 px
  xr = xr + (fabsf(xr) * 1e-3f + 0.01f);
  xl = xl - (fabsf(xl) * 1e-3f + 0.01f);
  const float px0 = ceilf(s.mx + xl - 0.5f), px1 = floorf(s.mx + xr - 0.5f);
  if (!(px0 <= px1) || !(px1 >= 0.0f)) return;
  const float lo = fmaxf(px0, 0.0f);
  const int tsh = 31 - __clz(tw);             // tile widths are powers of two
  const int t0 = (int)fminf(lo, 1e9f) >> tsh;
  const int t1 = ((int)fminf(px1, 1e9f) >> tsh) + 1;
  c0 = max(x0, t0);
  c1 = min(x1, t1);
  // skew cut over the tiles of this row (tile boxes: half extents tw/2, th/2)
  if (s.cut && c0 < c1) {
    const float hx = 0.5f * (float)tw, hy = 0.5f * (float)th;
    const float cy = (float)(row * th) + hy;
    const float base = skew_box_max(s.bx, s.by, hx, cy, s.mx, s.my, hx, hy);   // column 0
    const float step = s.bx * (float)tw;                                        // per column
    const float slack = 1e-3f * (1.0f + fabsf(base) + fabsf(s.need) + fabsf(step) * (float)c1);
    const float istep = __builtin_amdgcn_rcpf(step);
    if (step > 0.0f) {
      const float k = (s.need - base - slack) * istep;
      if (k > (float)c0) c0 = min(c1, (int)ceilf(fminf(k, 1e9f)));
    } else if (step < 0.0f) {
      const float k = (s.need - base - slack) * istep;   // columns <= k survive
      if (k < (float)(c1 - 1)) c1 = max(c0, (int)floorf(fmaxf(k, -1e9f)) + 1);
    } else if (base + slack < s.need) {
      c1 = c0;
    }
  }
  if (c1 < c0) c1 = c0;
}

// ---------------------------------------------------------------- wave ops
// Wave vote on a condition held as a lane mask: the ballot of the bool
// itself (the HIP __any / __all take an int, which costs a select and a
// compare per call to turn the mask into an int and back).  Lanes that are
// not active count as false for wave_any and as true for wave_all.
__device__ __forceinline__ bool wave_any(bool b) { return __builtin_amdgcn_ballot_w64(b) != 0ull; }
__device__ __forceinline__ bool wave_all(bool b) { return __builtin_amdgcn_ballot_w64(!b) == 0ull; }

// v of the lane that the DPP control CTRL selects (0 where none).
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_src(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, false));
}

// Inclusive prefix sum over the 64 lanes of the wave: within each row of 16
// by row shifts of 1, 2, 4 and 8, then the last lane of row 0 (of row 2) is
// broadcast into row 1 (row 3), and the last lane of row 1 into rows 2 and
// 3.  Lanes a DPP step has no source for add 0.  All 64 lanes must be
// active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}

// Inclusive prefix OR over the 64 lanes of the wave, by the same steps as
// wave_incl_scan.  All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_or(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}

// Inclusive prefix maximum over the 64 lanes of the wave (unsigned; lanes a
// DPP step has no source for take 0), by the same steps as wave_incl_scan.
// All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return v;
}

// Transposing sum over each 16-lane row of N <= 16 values per lane (missing
// values are 0): afterwards lane l of a row holds the row's sum of value
// l & 15.  Four butterfly steps halve the values per lane; at step h a lane
// keeps the half selected by its lane bit h and adds the partner's copy of
// that half, the partner being the lane DPP pairs it with (row mirror, half
// mirror, quad reversal, quad swap), which has the other bit h and holds the
// same set of values.  All 64 lanes must be active.
template <int N>
__device__ __forceinline__ float row_transpose_sum(const float (&g)[N], int lane) {
  static_assert(N <= 16, "at most 16 values per lane");
  float v16[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v16[k] = k < N ? g[k] : 0.0f;
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
  float v8[8], v4[4], v2[2];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    v8[k] = (b3 ? v16[k + 8] : v16[k]) + dpp_src<0x140>(b3 ? v16[k] : v16[k + 8]);   // row_mirror
#pragma unroll
  for (int k = 0; k < 4; ++k)
    v4[k] = (b2 ? v8[k + 4] : v8[k]) + dpp_src<0x141>(b2 ? v8[k] : v8[k + 4]);       // row_half_mirror
#pragma unroll
  for (int k = 0; k < 2; ++k)
    v2[k] = (b1 ? v4[k + 2] : v4[k]) + dpp_src<0x1B>(b1 ? v4[k] : v4[k + 2]);        // quad_perm [3,2,1,0]
  return (b0 ? v2[1] : v2[0]) + dpp_src<0xB1>(b0 ? v2[0] : v2[1]);                   // quad_perm [1,0,3,2]
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------- SH
// Real spherical harmonics up to degree 3 (3DGS ordering m = -l..l, sin terms
// for m < 0, Condon-Shortley phase), unit direction (x, y, z).
constexpr float SH_C0 = 0.28209479177387814f;
constexpr float SH_C1 = 0.4886025119029199f;
constexpr float SH_C2[5] = {1.0925484305920792f, -1.0925484305920792f, 0.31539156525252005f,
                            -1.0925484305920792f, 0.5462742152960396f};
constexpr float SH_C3[7] = {-0.5900435899266435f, 2.890611442640554f, -0.4570457994644658f,
                            0.3731763325901154f, -0.4570457994644658f, 1.445305721320277f,
                            -0.5900435899266435f};

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = SH_C0;
  if (DEG > 0) {
    Y[1] = -SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = -SH_C1 * x;
  }
  if (DEG > 1) {
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_C2[0] * x * y;
    Y[5] = SH_C2[1] * y * z;
    Y[6] = SH_C2[2] * (2.0f * zz - xx - yy);
    Y[7] = SH_C2[3] * x * z;
    Y[8] = SH_C2[4] * (xx - yy);
    if (DEG > 2) {
      Y[9] = SH_C3[0] * y * (3.0f * xx - yy);
      Y[10] = SH_C3[1] * x * y * z;
      Y[11] = SH_C3[2] * y * (4.0f * zz - xx - yy);
      Y[12] = SH_C3[3] * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = SH_C3[4] * x * (4.0f * zz - xx - yy);
      Y[14] = SH_C3[5] * z * (xx - yy);
      Y[15] = SH_C3[6] * x * (xx - 3.0f * yy);
    }
  }
}

// Gradient of sum_k w[k] Y_k(x,y,z) w.r.t. (x, y, z) of the polynomial forms
// above (the caller projects it onto the tangent plane of the unit sphere).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* w,
                                              float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (DEG > 0) {
    gy += -SH_C1 * w[1];
    gz += SH_C1 * w[2];
    gx += -SH_C1 * w[3];
  }
  if (DEG > 1) {
    float xx = x * x, yy = y * y, zz = z * z;
    gx += SH_C2[0] * y * w[4];
    gy += SH_C2[0] * x * w[4];
    gy += SH_C2[1] * z * w[5];
    gz += SH_C2[1] * y * w[5];
    gx += SH_C2[2] * (-2.0f * x) * w[6];
    gy += SH_C2[2] * (-2.0f * y) * w[6];
    gz += SH_C2[2] * (4.0f * z) * w[6];
    gx += SH_C2[3] * z * w[7];
    gz += SH_C2[3] * x * w[7];
    gx += SH_C2[4] * (2.0f * x) * w[8];
    gy += SH_C2[4] * (-2.0f * y) * w[8];
    if (DEG > 2) {
      // Y9 = C y (3xx - yy)
      gx += SH_C3[0] * 6.0f * x * y * w[9];
      gy += SH_C3[0] * (3.0f * xx - 3.0f * yy) * w[9];
      // Y10 = C x y z
      gx += SH_C3[1] * y * z * w[10];
      gy += SH_C3[1] * x * z * w[10];
      gz += SH_C3[1] * x * y * w[10];
      // Y11 = C y (4zz - xx - yy)
      gx += SH_C3[2] * (-2.0f * x * y) * w[11];
      gy += SH_C3[2] * (4.0f * zz - xx - 3.0f * yy) * w[11];
      gz += SH_C3[2] * (8.0f * y * z) * w[11];
      // Y12 = C z (2zz - 3xx - 3yy)
      gx += SH_C3[3] * (-6.0f * x * z) * w[12];
      gy += SH_C3[3] * (-6.0f * y * z) * w[12];
      gz += SH_C3[3] * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
      // Y13 = C x (4zz - xx - yy)
      gx += SH_C3[4] * (4.0f * zz - 3.0f * xx - yy) * w[13];
      gy += SH_C3[4] * (-2.0f * x * y) * w[13];
      gz += SH_C3[4] * (8.0f * x * z) * w[13];
      // Y14 = C z (xx - yy)
      gx += SH_C3[5] * (2.0f * x * z) * w[14];
      gy += SH_C3[5] * (-2.0f * y * z) * w[14];
      gz += SH_C3[5] * (xx - yy) * w[14];
      // Y15 = C x (xx - 3yy)
      gx += SH_C3[6] * (3.0f * xx - 3.0f * yy) * w[15];
      gy += SH_C3[6] * (-6.0f * x * y) * w[15];
    }
  }
}

// ---------------------------------------------------------------- camera
__device__ __forceinline__ int find_view(const sgs_camera* cams, int n_views, int tile) {
  int v = 0;
  for (int k = 1; k < n_views; ++k)
    if (tile >= cams[k].tile_base) v = k;
  return v;
}

// Spreads consecutive workgroups over tile bands so that the tiles one XCD
// (chiplet, own L2) works on are neighbours: workgroups are dispatched to the
// 8 XCDs round-robin, so workgroup b runs on XCD b % 8.
__device__ __forceinline__ int xcd_tile(int b, int total_tiles, int n_blocks) {
  const int per = n_blocks >> 3;      // n_blocks is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

}  // namespace sgs
