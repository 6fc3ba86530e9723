// ADAM Step of Algorithm 2 over every factor entry in one launch:
//   u <- b1 u + (1-b1) g ; v <- b2 v + (1-b2) g^2 ;
//   a <- max(a - alpha~ u / (sqrt(v) + eps), l)
// alpha~ = alpha sqrt(1-b2^n)/(1-b1^n) is formed on the host in FP64 from the
// stream's global iteration index (n = i + 1).
#include "common.hpp"

namespace gcp {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_adam(int64_t n, T* __restrict__ a, const T* __restrict__ g,
                                              T* __restrict__ u, T* __restrict__ v, T alpha_t, T b1, T b2,
                                              T eps, T lower) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T gi = g[i];
    T ui = b1 * u[i] + (T(1) - b1) * gi;
    T vi = b2 * v[i] + (T(1) - b2) * gi * gi;
    u[i] = ui;
    v[i] = vi;
    T ai = a[i] - alpha_t * ui / (sqrt(vi) + eps);
    a[i] = ai < lower ? lower : ai;   // keeps a NaN visible
  }
}

}  // namespace

hipError_t adam_run(int dtype, int64_t n, void* a, const void* g, void* u, void* v, double alpha_t, double beta1,
                    double beta2, double eps, double lower, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>(2048, (n + 255) / 256);
  if (dtype)
    hipLaunchKernelGGL(k_adam<double>, dim3(blocks), dim3(256), 0, st, n, static_cast<double*>(a),
                       static_cast<const double*>(g), static_cast<double*>(u), static_cast<double*>(v), alpha_t,
                       beta1, beta2, eps, lower);
  else
    hipLaunchKernelGGL(k_adam<float>, dim3(blocks), dim3(256), 0, st, n, static_cast<float*>(a),
                       static_cast<const float*>(g), static_cast<float*>(u), static_cast<float*>(v),
                       (float)alpha_t, (float)beta1, (float)beta2, (float)eps,
                       lower == -INFINITY ? -INFINITY : (float)lower);
  return hipGetLastError();
}

}  // namespace gcp
