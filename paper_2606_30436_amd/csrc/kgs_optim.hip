// Adam over a parameter vector of the map (the sliding-window optimisation of
// Sec. 3.2 updates the map by gradient steps; the paper names no optimiser, and
// Adam with bias correction is the reading).  One pass over theta, m, v and the
// gradient: HBM bound, 16 bytes read and 12 written per parameter.
#include <cmath>

#include "kgs_internal.h"

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

kgs_status kgs_launch_adam(float* theta, float* m, float* v, const float* g, int64_t n, int32_t step, float lr,
                           float b1, float b2, float eps, hipStream_t st) {
  if (n == 0) return KGS_OK;
  // bias corrections on the host in FP64 (1 - b2^t is small for early steps and would cancel in FP32)
  const float c1 = (float)(1.0 - pow((double)b1, (double)step)), c2 = (float)(1.0 - pow((double)b2, (double)step));
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_adam, dim3(grid), dim3(256), 0, st, theta, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return kgs_check_launch();
}
