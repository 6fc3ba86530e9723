// Evaluation metrics of Section 6: the sum of squares of a dense slice (the
// denominator of the local and global reconstruction losses, eq.
// local_loss), and the inner products behind the K-tensor congruence score
// (column norms of both K-tensors and the cross products a_r' b_q of every
// mode).  All sums are in FP64 and in a fixed order.
#include "solvers.hpp"

namespace gcp {
namespace {

constexpr int kMetThreads = 256;
constexpr int kMetBlocks = 1024;

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kMetThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

template <typename T>
__global__ void __launch_bounds__(kMetThreads) k_sumsq_part(const T* __restrict__ X, int64_t n, double* part) {
  __shared__ double red[kMetThreads];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)kMetThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kMetThreads) {
    const double x = (double)X[e];
    acc += x * x;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kMetThreads) k_sumsq_final(const double* part, int nblk, double* out) {
  __shared__ double red[kMetThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kMetThreads) acc += part[b];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) *out = t;
}

// Block (k, c): c < Ra: column c of A^(k) against every column of B^(k) and
// itself; c >= Ra: the norm of column c - Ra of B^(k).
template <typename T>
__global__ void __launch_bounds__(kMetThreads) k_cross(const T* A0, const T* A1, const T* A2, const T* B0,
                                                       const T* B1, const T* B2, int I0, int I1, int I2, int Ra,
                                                       int Rb, double* out) {
  __shared__ double red[kMetThreads];
  const int k = blockIdx.y;
  const int c = blockIdx.x;
  const T* A = k == 0 ? A0 : (k == 1 ? A1 : A2);
  const T* B = k == 0 ? B0 : (k == 1 ? B1 : B2);
  const int I = k == 0 ? I0 : (k == 1 ? I1 : I2);
  double* C = out + (size_t)k * Ra * Rb;             // [3][Ra][Rb]
  double* Na = out + (size_t)3 * Ra * Rb + k * Ra;    // [3][Ra]
  double* Nb = out + (size_t)3 * Ra * Rb + 3 * Ra + k * Rb;  // [3][Rb]
  if (c >= Ra) {
    const int q = c - Ra;
    double acc = 0.0;
    for (int i = threadIdx.x; i < I; i += kMetThreads) {
      const double b = (double)B[(size_t)i * Rb + q];
      acc += b * b;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) Nb[q] = t;
    return;
  }
  double acc = 0.0;
  for (int i = threadIdx.x; i < I; i += kMetThreads) {
    const double a = (double)A[(size_t)i * Ra + c];
    acc += a * a;
  }
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) Na[c] = t;
  for (int q = 0; q < Rb; ++q) {
    acc = 0.0;
    for (int i = threadIdx.x; i < I; i += kMetThreads)
      acc += (double)A[(size_t)i * Ra + c] * (double)B[(size_t)i * Rb + q];
    t = block_sum(acc, red);
    if (threadIdx.x == 0) C[(size_t)c * Rb + q] = t;
  }
}

template <typename T>
__global__ void k_add_scalar(T* p, double v) {
  *p = (T)((double)*p + v);
}

template <typename T>
__global__ void k_fill(T* p, int n, T v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

}  // namespace

hipError_t fill_run(int dtype, void* p, int n, double v, hipStream_t stream) {
  if (dtype)
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(256), 0, stream, static_cast<double*>(p), n, v);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(1), dim3(256), 0, stream, static_cast<float*>(p), n, (float)v);
  return hipGetLastError();
}

hipError_t scalar_add_run(int dtype, void* p, double v, hipStream_t stream) {
  if (dtype)
    hipLaunchKernelGGL(k_add_scalar<double>, dim3(1), dim3(1), 0, stream, static_cast<double*>(p), v);
  else
    hipLaunchKernelGGL(k_add_scalar<float>, dim3(1), dim3(1), 0, stream, static_cast<float*>(p), v);
  return hipGetLastError();
}

size_t metrics_ws_bytes() {
  return align_up((kMetBlocks + 1) * sizeof(double), 256) +
         align_up((size_t)(3 * kMaxRank * kMaxRank + 6 * kMaxRank) * sizeof(double), 256) +
         kMaxRank * sizeof(double);   // a row of ones (matrix slices' fixed mode of a reference K-tensor)
}

void* metrics_ones(void* ws) {
  return static_cast<char*>(ws) + metrics_ws_bytes() - kMaxRank * sizeof(double);
}

hipError_t sumsq_run(int dtype, const void* X, int64_t n, void* ws, double* out, hipStream_t stream) {
  double* part = static_cast<double*>(ws);
  const int nblk = (int)std::min<int64_t>(kMetBlocks, std::max<int64_t>(1, (n + kMetThreads - 1) / kMetThreads));
  if (dtype)
    hipLaunchKernelGGL(k_sumsq_part<double>, dim3(nblk), dim3(kMetThreads), 0, stream, static_cast<const double*>(X),
                       n, part);
  else
    hipLaunchKernelGGL(k_sumsq_part<float>, dim3(nblk), dim3(kMetThreads), 0, stream, static_cast<const float*>(X), n,
                       part);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(kMetThreads), 0, stream, part, nblk, out);
  return hipGetLastError();
}

namespace {
// out[row * I3 + i3] = bit i3 % 32 of word i3 / 32 of the row (rows of rpw words)
__global__ void __launch_bounds__(256) k_unpack_bits(const uint32_t* __restrict__ words, float* __restrict__ out,
                                                     int64_t rows, int I3, int rpw) {
  const int64_t n = rows * I3;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n; o += (int64_t)gridDim.x * 256) {
    const int64_t row = o / I3;
    const int i3 = (int)(o - row * I3);
    out[o] = (float)((words[row * rpw + (i3 >> 5)] >> (i3 & 31)) & 1u);
  }
}
}  // namespace

hipError_t unpack_bits_run(const void* words, float* out, int64_t rows, int I3, hipStream_t stream) {
  const int64_t n = rows * I3;
  const int blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_unpack_bits, dim3(blocks), dim3(256), 0, stream, static_cast<const uint32_t*>(words), out,
                     rows, I3, (I3 + 31) / 32);
  return hipGetLastError();
}

hipError_t cross_run(int dtype, const void* const* A, const void* const* B, const int* I, int Ra, int Rb, void* ws,
                     hipStream_t stream) {
  double* out = reinterpret_cast<double*>(static_cast<char*>(ws) + align_up((kMetBlocks + 1) * sizeof(double), 256));
  const dim3 grid(Ra + Rb, 3);
  if (dtype)
    hipLaunchKernelGGL(k_cross<double>, grid, dim3(kMetThreads), 0, stream, static_cast<const double*>(A[0]),
                       static_cast<const double*>(A[1]), static_cast<const double*>(A[2]),
                       static_cast<const double*>(B[0]), static_cast<const double*>(B[1]),
                       static_cast<const double*>(B[2]), I[0], I[1], I[2], Ra, Rb, out);
  else
    hipLaunchKernelGGL(k_cross<float>, grid, dim3(kMetThreads), 0, stream, static_cast<const float*>(A[0]),
                       static_cast<const float*>(A[1]), static_cast<const float*>(A[2]),
                       static_cast<const float*>(B[0]), static_cast<const float*>(B[1]),
                       static_cast<const float*>(B[2]), I[0], I[1], I[2], Ra, Rb, out);
  return hipGetLastError();
}

const double* cross_results(const void* ws) {
  return reinterpret_cast<const double*>(static_cast<const char*>(ws) +
                                         align_up((kMetBlocks + 1) * sizeof(double), 256));
}

}  // namespace gcp
