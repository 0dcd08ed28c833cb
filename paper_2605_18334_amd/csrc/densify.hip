// Densification step (Sec. "Depth-Aware Densification Strategy"): which
// Gaussians to clone or split from the accumulated screen-space and depth
// gradient statistics, and the new Gaussian set.
//
// Decision per Gaussian i (taken in float32):
//   selected = uv_sum / view_count >= tau_uv  or  z_max >= tau_z
//   split if selected and its largest log-scale > log(dense_scale), clone if
//   selected otherwise, keep if not selected.
// Output, in input order: a kept Gaussian once; a cloned one twice (two
// copies); a split one as its two children.  Children (the split along the
// largest axis e, with scales adjusted to the skew): the child scale along e
// is s_max / shrink, the other scales and every other attribute are the
// parent's; with Sigma the parent's covariance, delta = Sigma beta /
// sqrt(1 + beta^T Sigma beta) (and delta_c, Sigma_c of a child), the
// children sit at
//   mu + sqrt(2/pi) (delta - delta_c) +- a e,
//   a^2 = max(0, v - v_c),  v = s_max^2 - (2/pi) (e.delta)^2,
//   v_c = s_c^2 - (2/pi) (e.delta_c)^2,
// so that the pair (as skew-normal densities of weight 1/2) has the parent's
// mean and its variance along e.
//
// Three launches: decisions and per-block output counts; one block scans
// the counts; the emit kernel writes each Gaussian's outputs at its offset.
#include <math.h>

#include "sgs_dev.h"

namespace sgs {

constexpr int DN_T = 256;

struct DensArgs {
  sgs_params p;
  const float* uv_sum;
  const uint32_t* view_count;
  const float* z_max;
  float tau_uv, tau_z, log_dense, shrink;
  uint8_t* decision;
  uint32_t* block_out;    // [nb + 1]: per-block output counts, then their exclusive prefix
  sgs_densify_out out;
  uint32_t* n_out;        // [1]
};

__device__ __forceinline__ uint8_t decide(const DensArgs& a, int64_t i, int& kmax) {
  const int64_t n = a.p.n;
  const uint32_t c = a.view_count ? a.view_count[i] : 0u;
  const float avg = c ? a.uv_sum[i] / (float)c : 0.0f;
  const bool sel = (a.uv_sum && avg >= a.tau_uv) || (a.z_max && a.z_max[i] >= a.tau_z);
  float lmax = a.p.log_scale[i];
  kmax = 0;
  for (int k = 1; k < 3; ++k) {
    const float l = a.p.log_scale[k * n + i];
    if (l > lmax) {
      lmax = l;
      kmax = k;
    }
  }
  if (!sel) return 0;
  return lmax > a.log_dense ? 2 : 1;
}

__global__ void __launch_bounds__(DN_T) k_dens_decide(DensArgs a) {
  __shared__ uint32_t ws[DN_T / 64];
  const int64_t i = (int64_t)blockIdx.x * DN_T + threadIdx.x;
  uint32_t outs = 0;
  if (i < a.p.n) {
    int kmax;
    const uint8_t d = decide(a, i, kmax);
    a.decision[i] = d;
    outs = d ? 2u : 1u;
  }
  uint32_t s = outs;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < DN_T / 64; ++w) t += ws[w];
    a.block_out[blockIdx.x] = t;
  }
}

// Exclusive scan of nb counts in place; block_out[nb] and *n_out get the total.
__global__ void __launch_bounds__(1024) k_dens_scan(uint32_t* block_out, int64_t nb, uint32_t* n_out) {
  __shared__ uint32_t ws[16];
  __shared__ uint32_t s_carry;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t k = base + t;
    const uint32_t x = k < nb ? block_out[k] : 0u;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t e = inc - x + s_carry;
    for (int q = 0; q < w; ++q) e += ws[q];
    __syncthreads();
    if (k < nb) block_out[k] = e;
    if (t == 1023) s_carry = e + x;
    __syncthreads();
  }
  if (t == 0) {
    block_out[nb] = s_carry;
    *n_out = s_carry;
  }
}

__device__ __forceinline__ void put(const DensArgs& a, int64_t o, int64_t i, const float mean[3],
                                    const float ls[3]) {
  const int64_t n = a.p.n, cap = a.out.capacity;
  if (o >= cap) return;
  for (int k = 0; k < 3; ++k) {
    a.out.mean[k * cap + o] = mean[k];
    a.out.log_scale[k * cap + o] = ls[k];
    if (a.out.skew && a.p.skew) a.out.skew[k * cap + o] = a.p.skew[k * n + i];
    if (a.out.opa_dir && a.p.opa_dir) a.out.opa_dir[k * cap + o] = a.p.opa_dir[k * n + i];
  }
  for (int k = 0; k < 4; ++k) a.out.quat[k * cap + o] = a.p.quat[k * n + i];
  a.out.opa_logit[o] = a.p.opa_logit[i];
  if (a.out.opa2_logit && a.p.opa2_logit) a.out.opa2_logit[o] = a.p.opa2_logit[i];
  const int K3 = 3 * (a.p.sh_degree + 1) * (a.p.sh_degree + 1);
  for (int k = 0; k < K3; ++k) a.out.sh[(int64_t)k * cap + o] = a.p.sh[(int64_t)k * n + i];
  if (a.out.parent) a.out.parent[o] = (uint32_t)i;
}

// delta = Sigma beta / sqrt(1 + beta^T Sigma beta) with Sigma = R diag(s^2) R^T.
__device__ __forceinline__ void skew_delta(const float R[3][3], const float s[3], const float b[3],
                                           float d[3]) {
  float u[3];   // diag(s) R^T beta
  for (int c = 0; c < 3; ++c) u[c] = s[c] * (R[0][c] * b[0] + R[1][c] * b[1] + R[2][c] * b[2]);
  const float kappa = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float r = 1.0f / sqrtf(1.0f + kappa);
  for (int k = 0; k < 3; ++k) d[k] = r * (R[k][0] * s[0] * u[0] + R[k][1] * s[1] * u[1] + R[k][2] * s[2] * u[2]);
}

__global__ void __launch_bounds__(DN_T) k_dens_emit(DensArgs a) {
  __shared__ uint32_t ws[DN_T / 64];
  const int64_t n = a.p.n;
  const int64_t i = (int64_t)blockIdx.x * DN_T + threadIdx.x;
  const uint8_t d = i < n ? a.decision[i] : 0;
  const uint32_t outs = i < n ? (d ? 2u : 1u) : 0u;
  const uint32_t inc = wave_incl_scan(outs);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t e = inc - outs + a.block_out[blockIdx.x];
  for (int q = 0; q < w; ++q) e += ws[q];
  if (i >= n) return;
  float mean[3], ls[3];
  for (int k = 0; k < 3; ++k) {
    mean[k] = a.p.mean[k * n + i];
    ls[k] = a.p.log_scale[k * n + i];
  }
  if (d != 2) {
    put(a, e, i, mean, ls);
    if (d == 1) put(a, (int64_t)e + 1, i, mean, ls);
    return;
  }
  int kmax;
  decide(a, i, kmax);
  float qw = a.p.quat[i], qx = a.p.quat[n + i], qy = a.p.quat[2 * n + i], qz = a.p.quat[3 * n + i];
  const float iq = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  const float R[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                         {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                         {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
  float s[3], sc[3], b[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < 3; ++k) s[k] = expf(ls[k]);
  if (a.p.skew)
    for (int k = 0; k < 3; ++k) b[k] = a.p.skew[k * n + i];
  const float smax = s[kmax], sch = smax / a.shrink;
  for (int k = 0; k < 3; ++k) sc[k] = k == kmax ? sch : s[k];
  float dp[3], dc[3];
  skew_delta(R, s, b, dp);
  skew_delta(R, sc, b, dc);
  const float e3[3] = {R[0][kmax], R[1][kmax], R[2][kmax]};
  const float ep = e3[0] * dp[0] + e3[1] * dp[1] + e3[2] * dp[2];
  const float ec = e3[0] * dc[0] + e3[1] * dc[1] + e3[2] * dc[2];
  constexpr float TWO_OVER_PI = 0.63661977236758134f;
  constexpr float SQRT_TWO_OVER_PI = 0.79788456080286536f;
  const float v = smax * smax - TWO_OVER_PI * ep * ep;
  const float vc = sch * sch - TWO_OVER_PI * ec * ec;
  const float h = sqrtf(fmaxf(v - vc, 0.0f));
  float m0[3], m1[3], lc[3];
  for (int k = 0; k < 3; ++k) {
    const float c = mean[k] + SQRT_TWO_OVER_PI * (dp[k] - dc[k]);
    m0[k] = c + h * e3[k];
    m1[k] = c - h * e3[k];
    lc[k] = k == kmax ? logf(sch) : ls[k];
  }
  put(a, e, i, m0, lc);
  put(a, (int64_t)e + 1, i, m1, lc);
}

sgs_status launch_densify(const sgs_params* p, const float* uv_sum, const uint32_t* view_count,
                          const float* z_max, const sgs_densify_options* o, uint8_t* decision,
                          uint32_t* block_out, const sgs_densify_out* out, uint32_t* n_out,
                          hipStream_t s) {
  DensArgs a;
  a.p = *p;
  a.uv_sum = uv_sum;
  a.view_count = view_count;
  a.z_max = z_max;
  a.tau_uv = o->tau_uv;
  a.tau_z = o->tau_z;
  a.log_dense = (float)log((double)o->dense_scale);
  a.shrink = o->split_shrink;
  a.decision = decision;
  a.block_out = block_out;
  a.out = *out;
  a.n_out = n_out;
  const int64_t nb = (p->n + DN_T - 1) / DN_T;
  if (nb > 0) {
    k_dens_decide<<<(unsigned)nb, DN_T, 0, s>>>(a);
    SGS_LAUNCH_CHECK();
  }
  k_dens_scan<<<1, 1024, 0, s>>>(block_out, nb, n_out);
  SGS_LAUNCH_CHECK();
  if (nb > 0 && out->capacity > 0) {
    k_dens_emit<<<(unsigned)nb, DN_T, 0, s>>>(a);
    SGS_LAUNCH_CHECK();
  }
  return SGS_OK;
}

}  // namespace sgs
