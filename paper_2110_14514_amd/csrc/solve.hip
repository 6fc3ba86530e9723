// Least-squares temporal-weight solve for the Gaussian loss (Section 5: one
// least-squares solve replaces the SGD temporal solver of Algorithm 3).
//
// The temporal subproblem (eq. gcp_stream_temporal_problem) with
// f = (x-m)^2 and m = Z s is stationary where
//     (Gamma + mu/2 I) s = b,   Gamma = hadamard_k A^(k)^T A^(k),
//                               b = Z^T vec(X_t).
// Pass 1 streams X_t once and forms per-workgroup partials of b in FP32.
// Pass 2 (one workgroup) sums the partials in FP64, forms Gamma in FP64, and
// solves by an FP64 Cholesky factorisation in LDS; then s <- max(s, l).
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kPairChunk = 64;

constexpr int kGramRows = 64;   // factor rows per workgroup of the Gram partials

struct LsLayout {
  int nchunks, ygs;
  int gch[3];         // Gram row chunks per mode
  size_t gram_off;    // byte offset of the Gram partials (R x R doubles per chunk)
  size_t bytes;
};

LsLayout ls_layout(int I1, int I2, int I3, int R) {
  LsLayout L;
  L.nchunks = (int)(((size_t)I1 * I2 + kPairChunk - 1) / kPairChunk);
  L.ygs = (I3 + 255) / 256;
  const int I[3] = {I1, I2, I3};
  for (int k = 0; k < 3; ++k) L.gch[k] = (I[k] + kGramRows - 1) / kGramRows;
  L.gram_off = align_up((size_t)L.nchunks * L.ygs * R * sizeof(double), 256);
  L.bytes = L.gram_off + align_up((size_t)(L.gch[0] + L.gch[1] + L.gch[2]) * R * R * sizeof(double), 256);
  return L;
}

// b partials: workgroup (chunk of 64 (i1, i2) pairs, block of 256 i3):
// the chunk's products w = a1 * a2 are staged in LDS (zeros past R), thread
// i3 sums x * w over the chunk and scales by a3[i3] at the end.
template <typename T, int RT>
__global__ void __launch_bounds__(256) k_ls_b(const T* __restrict__ X, const T* __restrict__ A1,
                                              const T* __restrict__ A2, const T* __restrict__ A3,
                                              double* __restrict__ bp, int I1, int I2, int I3, int R) {
  __shared__ T w[kPairChunk][RT];
  __shared__ T sm[4][RT];
  const int chunk = blockIdx.x;
  const int i3 = blockIdx.y * 256 + threadIdx.x;
  const int p0 = chunk * kPairChunk;
  const int npairs = I1 * I2;                     // < 2^31 (checked at stream creation)
  const int np = min(kPairChunk, npairs - p0);
  for (int e = threadIdx.x; e < kPairChunk * RT; e += 256) {
    const int q = e / RT, j = e - (e / RT) * RT;
    T v = T(0);
    if (q < np && j < R) {
      const int p = p0 + q, i1 = p / I2, i2 = p - i1 * I2;
      v = A1[(size_t)i1 * R + j] * A2[(size_t)i2 * R + j];
    }
    w[q][j] = v;
  }
  __syncthreads();
  T acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc[j] = T(0);
  if (i3 < I3) {
    const T* xp = X + (size_t)p0 * I3 + i3;
    for (int q0 = 0; q0 < np; q0 += 8) {
      T x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = q0 + u < np ? xp[(size_t)(q0 + u) * I3] : T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (q0 + u >= np) break;
#pragma unroll
        for (int j = 0; j < RT; ++j) acc[j] += x[u] * w[q0 + u][j];
      }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j) acc[j] *= j < R ? A3[(size_t)i3 * R + j] : T(0);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < RT; ++j) {
    T v = acc[j];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) sm[wave][j] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < R) {
    int j = threadIdx.x;
    double v = (((double)sm[0][j] + (double)sm[1][j]) + (double)sm[2][j]) + (double)sm[3][j];
    bp[((size_t)chunk * gridDim.y + blockIdx.y) * R + j] = v;
  }
}

// Gram partials: workgroup b takes kGramRows rows of one factor (mode k,
// row chunk c) through LDS and writes sum_i A_k[i][r] A_k[i][c] (FP64) for
// the lower triangle; thread tid owns entries tid, tid + 256, ...
template <typename T>
__global__ void __launch_bounds__(256) k_ls_gram(const T* __restrict__ A1, const T* __restrict__ A2,
                                                 const T* __restrict__ A3, int I1, int I2, int I3, int R, int c1,
                                                 int c2, double* __restrict__ gp) {
  __shared__ T st[kGramRows][kMaxRank + 1];
  const int b = blockIdx.x;
  const int k = b < c1 ? 0 : (b < c1 + c2 ? 1 : 2);
  const int c = b - (k == 0 ? 0 : (k == 1 ? c1 : c1 + c2));
  const T* A = k == 0 ? A1 : (k == 1 ? A2 : A3);
  const int I = k == 0 ? I1 : (k == 1 ? I2 : I3);
  const int i0 = c * kGramRows, nr = min(kGramRows, I - i0);
  for (int e = threadIdx.x; e < nr * R; e += 256) st[e / R][e % R] = A[(size_t)i0 * R + e];
  __syncthreads();
  for (int idx = threadIdx.x; idx < R * R; idx += 256) {
    const int r = idx / R, cc = idx % R;
    if (cc > r) continue;
    double acc = 0.0;
    for (int i = 0; i < nr; ++i) acc += (double)st[i][r] * (double)st[i][cc];
    gp[(size_t)b * R * R + idx] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ls_solve(const double* __restrict__ bp, int nparts,
                                                  const double* __restrict__ gp, int3 gch3, int R, double half_mu,
                                                  double lower, T* __restrict__ s_out, int* status) {
  __shared__ double L[kMaxRank][kMaxRank + 1];
  __shared__ double b[kMaxRank];
  __shared__ int bad;
  const int gch[3] = {gch3.x, gch3.y, gch3.z};
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  // b = sum of partials in a fixed order: thread tid = q RP + j sums parts
  // q, q + 256/RP, ... of column j, then a fixed tree over q
  {
    __shared__ double red[256];
    const int RP = R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
    const int groups = 256 / RP, j = tid % RP, q = tid / RP;
    double s = 0.0;
    if (j < R)
      for (int c0 = q; c0 < nparts; c0 += 8 * groups) {
        double v[8];   // eight loads in flight, added in part order
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + u * groups;
          v[u] = c < nparts ? bp[(size_t)c * R + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
    red[tid] = s;
    __syncthreads();
    for (int w = groups / 2; w >= 1; w >>= 1) {
      if (q < w) red[tid] += red[tid + w * RP];
      __syncthreads();
    }
    if (tid < R) b[tid] = red[tid];
  }
  // Gamma[r][c] = prod_k sum_i A_k[i][r] A_k[i][c] (FP64, lower triangle):
  // each mode's chunk partials added in chunk order
  for (int idx = tid; idx < R * R; idx += 256) {
    const int r = idx / R, c = idx % R;
    if (c > r) continue;
    double g = 1.0;
    int b0 = 0;
    for (int k = 0; k < 3; ++k) {
      double d = 0.0;
      for (int ch = 0; ch < gch[k]; ++ch) d += gp[(size_t)(b0 + ch) * R * R + idx];
      b0 += gch[k];
      g *= d;
    }
    L[r][c] = g + (r == c ? half_mu : 0.0);
  }
  __syncthreads();
  // right-looking Cholesky, lower triangle in place
  for (int k = 0; k < R; ++k) {
    if (tid == 0) {
      double d = L[k][k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        d = 1.0;
      }
      L[k][k] = sqrt(d);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < R; i += 256) L[i][k] /= L[k][k];
    __syncthreads();
    for (int idx = tid; idx < R * R; idx += 256) {
      int i = idx / R, j = idx % R;
      if (j > k && i >= j) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  if (tid == 0) {
    // L y = b ; L^T s = y
    for (int i = 0; i < R; ++i) {
      double v = b[i];
      for (int j = 0; j < i; ++j) v -= L[i][j] * b[j];
      b[i] = v / L[i][i];
    }
    for (int i = R - 1; i >= 0; --i) {
      double v = b[i];
      for (int j = i + 1; j < R; ++j) v -= L[j][i] * b[j];
      b[i] = v / L[i][i];
    }
    if (bad) atomicOr(status, (int)kStatusPivot);
  }
  __syncthreads();
  for (int j = tid; j < R; j += 256) {
    double v = bad ? (double)NAN : fmax(b[j], lower);
    s_out[j] = (T)v;
  }
}

template <typename T, int RT>
hipError_t run_ls(int I1, int I2, int I3, int R, const void* X, const void* const* A, double mu, double lower,
                  void* s_out, void* scratch, int* status, hipStream_t st) {
  LsLayout L = ls_layout(I1, I2, I3, R);
  double* bp = static_cast<double*>(scratch);
  hipLaunchKernelGGL((k_ls_b<T, RT>), dim3(L.nchunks, L.ygs), dim3(256), 0, st, static_cast<const T*>(X),
                     static_cast<const T*>(A[0]), static_cast<const T*>(A[1]), static_cast<const T*>(A[2]), bp,
                     I1, I2, I3, R);
  double* gp = reinterpret_cast<double*>(static_cast<char*>(scratch) + L.gram_off);
  hipLaunchKernelGGL((k_ls_gram<T>), dim3(L.gch[0] + L.gch[1] + L.gch[2]), dim3(256), 0, st,
                     static_cast<const T*>(A[0]), static_cast<const T*>(A[1]), static_cast<const T*>(A[2]), I1, I2,
                     I3, R, L.gch[0], L.gch[1], gp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ls_solve<T>), dim3(1), dim3(256), 0, st, bp, L.nchunks * L.ygs, gp,
                     make_int3(L.gch[0], L.gch[1], L.gch[2]), R, 0.5 * mu, lower, static_cast<T*>(s_out), status);
  return hipGetLastError();
}

template <typename T>
hipError_t run_ls_t(int I1, int I2, int I3, int R, const void* X, const void* const* A, double mu, double lower,
                    void* s_out, void* scratch, int* status, hipStream_t st) {
  if (R <= 8) return run_ls<T, 8>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st);
  if (R <= 16) return run_ls<T, 16>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st);
  if (R <= 32) return run_ls<T, 32>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st);
  return run_ls<T, 64>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st);
}

}  // namespace

size_t ls_scratch_bytes(int I1, int I2, int I3, int R) { return ls_layout(I1, I2, I3, R).bytes; }

hipError_t ls_solve_run(int I1, int I2, int I3, int R, int dtype, const void* X, const void* const* A, double mu,
                        double lower, void* s_out, void* scratch, int* status, hipStream_t st) {
  return dtype ? run_ls_t<double>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st)
               : run_ls_t<float>(I1, I2, I3, R, X, A, mu, lower, s_out, scratch, status, st);
}

}  // namespace gcp
