// Adam update of the Gaussian parameters (the optimiser of the photometric
// training loop, Sec. "Preliminary of 3D Gaussian Splatting": attributes are
// optimised by gradient descent on a photometric loss).  Two launches per
// step, both graph-capturable: one thread advances the step counter and the
// bias corrections in device memory, then one grid updates every parameter
// group (blockIdx.y = group).
#include "sgs_dev.h"

namespace sgs {

struct AdamGroups {
  sgs_adam_group g[SGS_ADAM_MAX_GROUPS];
};

// state: [0] step count t, [1] 1 / (1 - beta1^t), [2] 1 / (1 - beta2^t)
__global__ void k_adam_tick(float* state, float beta1, float beta2) {
  const float t = state[0] + 1.0f;
  state[0] = t;
  state[1] = 1.0f / (1.0f - powf(beta1, t));
  state[2] = 1.0f / (1.0f - powf(beta2, t));
}

__global__ void __launch_bounds__(256) k_adam(AdamGroups gs, const float* __restrict__ state,
                                              float beta1, float beta2, float eps) {
  const sgs_adam_group& g = gs.g[blockIdx.y];
  const float c1 = state[1], c2 = state[2];
  const float lr = g.lr;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * 256) {
    const float gr = g.grad[i];
    const float m = fmaf(beta1, g.m1[i], (1.0f - beta1) * gr);
    const float v = fmaf(beta2, g.m2[i], (1.0f - beta2) * gr * gr);
    g.m1[i] = m;
    g.m2[i] = v;
    g.param[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
  }
}

sgs_status launch_adam(const sgs_adam_group* groups, int32_t n_groups, float* state, float beta1,
                       float beta2, float eps, hipStream_t s) {
  AdamGroups a = {};
  int64_t nmax = 0;
  for (int k = 0; k < n_groups; ++k) {
    a.g[k] = groups[k];
    nmax = groups[k].n > nmax ? groups[k].n : nmax;
  }
  k_adam_tick<<<1, 1, 0, s>>>(state, beta1, beta2);
  SGS_LAUNCH_CHECK();
  if (nmax == 0) return SGS_OK;
  const int64_t blocks = (nmax + 255) / 256;
  k_adam<<<dim3((unsigned)(blocks < 4096 ? blocks : 4096), (unsigned)n_groups), 256, 0, s>>>(
      a, state, beta1, beta2, eps);
  SGS_LAUNCH_CHECK();
  return SGS_OK;
}

}  // namespace sgs
