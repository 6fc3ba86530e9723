// Four-way slices (d = 4) through merged modes.  With entry (i3, i4) stored
// as entry i3 I4 + i4 of an I1 x I2 x (I3 I4) slice, the CP model of
// Section 2.1 is the three-way model whose third factor has the rows
// A3[i3] * A4[i4] (a Khatri-Rao row), so the three-way kernels evaluate the
// objective and the first two gradients unchanged.  By the chain rule the
// merged mode's gradient G34 gives
//   G3[i3, j] = sum_i4 G34[i3 I4 + i4, j] A4[i4, j],
//   G4[i4, j] = sum_i3 G34[i3 I4 + i4, j] A3[i3, j],
// and the regulariser of Section 4.1 is taken on A3 and A4 themselves (the
// kernels run with none on the merged mode).
#include "solvers.hpp"

namespace gcp {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_kr_merge(const T* __restrict__ A3, const T* __restrict__ A4, int I3, int I4,
                                                  int R, T* __restrict__ out) {
  const int64_t n = (int64_t)I3 * I4 * R;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n; o += (int64_t)gridDim.x * 256) {
    const int64_t row = o / R;
    const int j = (int)(o - row * R);
    const int i3 = (int)(row / I4), i4 = (int)(row - (int64_t)i3 * I4);
    out[o] = A3[(int64_t)i3 * R + j] * A4[(int64_t)i4 * R + j];
  }
}

// One thread per output entry (mode 3 rows first, then mode 4), summing the
// merged rows in index order with compensation: the result does not depend
// on scheduling.
template <typename T>
__global__ void __launch_bounds__(256) k_project(const T* __restrict__ G34, const T* __restrict__ A3,
                                                 const T* __restrict__ A4, int I3, int I4, int R, T lam,
                                                 const T* __restrict__ gscale, T* __restrict__ G3,
                                                 T* __restrict__ G4, int* status) {
  const int64_t n3 = (int64_t)I3 * R, n4 = (int64_t)I4 * R;
  const T sc = gscale ? gscale[0] : T(1);
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n3 + n4; o += (int64_t)gridDim.x * 256) {
    Kahan<T> k;
    T out;
    if (o < n3) {
      const int i3 = (int)(o / R), j = (int)(o - (int64_t)i3 * R);
      for (int i4 = 0; i4 < I4; ++i4) k.add(G34[((int64_t)i3 * I4 + i4) * R + j] * A4[(int64_t)i4 * R + j]);
      out = k.s + sc * lam * A3[o];
      G3[o] = out;
    } else {
      const int64_t e = o - n3;
      const int i4 = (int)(e / R), j = (int)(e - (int64_t)i4 * R);
      for (int i3 = 0; i3 < I3; ++i3) k.add(G34[((int64_t)i3 * I4 + i4) * R + j] * A3[(int64_t)i3 * R + j]);
      out = k.s + sc * lam * A4[e];
      G4[e] = out;
    }
    if (!isfinite(out)) atomicOr(status, (int)kStatusNonFinite);
  }
}

// *loss += lam/2 (||A3||^2 + ||A4||^2), one workgroup
template <typename T>
__global__ void __launch_bounds__(256) k_reg_add(T* loss, const T* __restrict__ A3, int64_t n3,
                                                 const T* __restrict__ A4, int64_t n4, T lam) {
  __shared__ T red[256];
  Kahan<T> k;
  for (int64_t o = threadIdx.x; o < n3; o += 256) k.add(A3[o] * A3[o]);
  for (int64_t o = threadIdx.x; o < n4; o += 256) k.add(A4[o] * A4[o]);
  red[threadIdx.x] = k.s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] += T(0.5) * lam * red[0];
}

int grid_of(int64_t n) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

hipError_t kr_merge_run(int dtype, const void* A3, const void* A4, int I3, int I4, int R, void* out,
                        hipStream_t stream) {
  const int g = grid_of((int64_t)I3 * I4 * R);
  if (dtype)
    hipLaunchKernelGGL(k_kr_merge<double>, dim3(g), dim3(256), 0, stream, static_cast<const double*>(A3),
                       static_cast<const double*>(A4), I3, I4, R, static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_kr_merge<float>, dim3(g), dim3(256), 0, stream, static_cast<const float*>(A3),
                       static_cast<const float*>(A4), I3, I4, R, static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t merged_project_run(int dtype, const void* G34, const void* A3, const void* A4, int I3, int I4, int R,
                              double lam, const void* gscale, void* G3, void* G4, int* status, hipStream_t stream) {
  const int g = grid_of((int64_t)(I3 + I4) * R);
  if (dtype)
    hipLaunchKernelGGL(k_project<double>, dim3(g), dim3(256), 0, stream, static_cast<const double*>(G34),
                       static_cast<const double*>(A3), static_cast<const double*>(A4), I3, I4, R, lam,
                       static_cast<const double*>(gscale), static_cast<double*>(G3), static_cast<double*>(G4),
                       status);
  else
    hipLaunchKernelGGL(k_project<float>, dim3(g), dim3(256), 0, stream, static_cast<const float*>(G34),
                       static_cast<const float*>(A3), static_cast<const float*>(A4), I3, I4, R, (float)lam,
                       static_cast<const float*>(gscale), static_cast<float*>(G3), static_cast<float*>(G4), status);
  return hipGetLastError();
}

hipError_t merged_reg_run(int dtype, void* loss, const void* A3, int64_t n3, const void* A4, int64_t n4, double lam,
                          hipStream_t stream) {
  if (dtype)
    hipLaunchKernelGGL(k_reg_add<double>, dim3(1), dim3(256), 0, stream, static_cast<double*>(loss),
                       static_cast<const double*>(A3), n3, static_cast<const double*>(A4), n4, lam);
  else
    hipLaunchKernelGGL(k_reg_add<float>, dim3(1), dim3(256), 0, stream, static_cast<float*>(loss),
                       static_cast<const float*>(A3), n3, static_cast<const float*>(A4), n4, (float)lam);
  return hipGetLastError();
}

}  // namespace gcp
