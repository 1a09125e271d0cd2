// World->local instance records composed in float64 (Eq. 7, rigid map
// G(q) = s R q + T; rays are moved into canonical space).
#include <hip/hip_runtime.h>

#include "launch.h"

namespace nedf {
namespace {

__global__ void k_compose(const double* G, int n, float* w2l) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* g = G + 13 * size_t(i);
  const double s = g[12];
  const double inv_s = 1.0 / s;
  float* out = w2l + 16 * size_t(i);
  // R^T (row r of R^T is column r of R)
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[3 * r + c] = float(g[3 * c + r]);
  for (int r = 0; r < 3; ++r) {
    const double rt_t = g[0 * 3 + r] * g[9] + g[1 * 3 + r] * g[10] + g[2 * 3 + r] * g[11];
    out[9 + r] = float(-rt_t * inv_s);
  }
  out[12] = float(s);
  out[13] = float(inv_s);
  out[14] = 0.0f;
  out[15] = 0.0f;
}

}  // namespace

hipError_t launch_compose_transforms(const double* G, int32_t n, float* w2l, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose, dim3((n + 127) / 128), dim3(128), 0, s, G, n, w2l);
  return hipGetLastError();
}

}  // namespace nedf
