// Model-difference history term of eq. gcp_stream_problem_2 (Section 4.1)
// and its factor gradient, the history part of eq. spatial_gcp_grad
// (Section 4.2).  The window keeps only the weights s_h; the term compares
// the CP models of the previous step's factors Abar and of the current
// factors A, both with weight s_h:
//
//   F_hist = 1/2 sum_h w_h ||[[Abar; s_h]] - [[A; s_h]]||_F^2
//          = 1/2 <S_w, (*_k Abar_k' Abar_k) - 2 (*_k Abar_k' A_k) + (*_k A_k' A_k)>
//   dF_hist/dA_k = A_k B_k - Abar_k C_k,
//   B_k = (*_{l != k} A_l' A_l) o S_w,  C_k = (*_{l != k} Abar_l' A_l) o S_w,
//   S_w = sum_h w_h s_h s_h'
//
// (* and o: Hadamard products of R x R matrices; the closed forms follow from
// ||[[A; s]]||^2 = s' (*_k A_k' A_k) s and from diag(s) G diag(s) = G o s s').
// Every sum is formed in FP64 in a fixed order: the terms nearly cancel when
// the factors move little, and the results are bitwise repeatable.
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kHistThreads = 256;

// Offsets (in doubles) inside the history workspace.
__host__ __device__ inline size_t gram_off(int kind, int k, int R) { return (size_t)(3 * kind + k) * R * R; }
__host__ __device__ inline size_t b_off(int k, int R) { return (size_t)(9 + k) * R * R; }
__host__ __device__ inline size_t c_off(int k, int R) { return (size_t)(12 + k) * R * R; }

template <typename T>
struct HistArgs {
  const T* A[3];
  const T* Ab[3];
  const T* shist;
  T* G[3];
  T* loss;
  const T* gscale;
  double* ws;
  int* status;
  const int64_t* stamps;   // device, t_h of each window slot
  int64_t t;
  double w, theta;
  int I[3];
  int R, nwin, want;
};

// The window's weights w_h = w theta^(t - t_h) from the device-held slot
// stamps, into the workgroup's LDS (every thread of the one workgroup).
template <typename T>
__device__ void window_weights(const HistArgs<T>& a, double* cw) {
  for (int h = threadIdx.x; h < a.nwin; h += kHistThreads) cw[h] = a.w * pow(a.theta, (double)(a.t - a.stamps[h]));
  __syncthreads();
}

// Row i of the Gram matrix X_k' Y_k (kind 0: A'A, 1: Abar'A, 2: Abar'Abar).
// The workgroup's threads are (column j, row chunk c) with RP >= R columns
// (a power of two) and 256 / RP chunks; chunk c takes rows c, c + nc, ...
// with four independent partial sums (loads in flight), and the chunks are
// added in order.
template <typename T>
__global__ void __launch_bounds__(kHistThreads) hist_gram(HistArgs<T> a) {
  __shared__ double part[kHistThreads];
  const int i = blockIdx.x;
  const int kind = blockIdx.y / 3, k = blockIdx.y % 3;
  const T* X = kind == 0 ? a.A[k] : a.Ab[k];
  const T* Y = kind == 2 ? a.Ab[k] : a.A[k];
  const int R = a.R, n = a.I[k];
  int RP = 1;
  while (RP < R) RP <<= 1;
  const int nc = kHistThreads / RP;
  const int j = threadIdx.x % RP, c = threadIdx.x / RP;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (j < R) {
    int r = c;
    for (; r + 3 * nc < n; r += 4 * nc) {
      s0 += (double)X[(size_t)r * R + i] * (double)Y[(size_t)r * R + j];
      s1 += (double)X[(size_t)(r + nc) * R + i] * (double)Y[(size_t)(r + nc) * R + j];
      s2 += (double)X[(size_t)(r + 2 * nc) * R + i] * (double)Y[(size_t)(r + 2 * nc) * R + j];
      s3 += (double)X[(size_t)(r + 3 * nc) * R + i] * (double)Y[(size_t)(r + 3 * nc) * R + j];
    }
    for (; r < n; r += nc) s0 += (double)X[(size_t)r * R + i] * (double)Y[(size_t)r * R + j];
  }
  part[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (c == 0 && j < R) {
    double t = 0.0;
    for (int cc = 0; cc < nc; ++cc) t += part[cc * RP + j];
    a.ws[gram_off(kind, k, R) + (size_t)i * R + j] = t;
  }
}

// S_w, the matrices B_k and C_k, and the objective term (added to the loss).
template <typename T>
__global__ void __launch_bounds__(kHistThreads) hist_combine(HistArgs<T> a) {
  __shared__ double red[kHistThreads];
  const int R = a.R;
  const double* P = a.ws + gram_off(0, 0, R);
  const double* Q = a.ws + gram_off(1, 0, R);
  const double* O = a.ws + gram_off(2, 0, R);
  const size_t RR = (size_t)R * R;
  __shared__ double cw[kMaxWindowModel];
  window_weights(a, cw);
  double f = 0.0;
  for (int e = threadIdx.x; e < R * R; e += kHistThreads) {
    const int i = e / R, j = e - (e / R) * R;
    double sw = 0.0;
    for (int h = 0; h < a.nwin; ++h) sw += cw[h] * (double)a.shist[(size_t)h * R + i] * (double)a.shist[(size_t)h * R + j];
    const double p0 = P[e], p1 = P[RR + e], p2 = P[2 * RR + e];
    const double q0 = Q[e], q1 = Q[RR + e], q2 = Q[2 * RR + e];
    const double o0 = O[e], o1 = O[RR + e], o2 = O[2 * RR + e];
    a.ws[b_off(0, R) + e] = sw * (p1 * p2);
    a.ws[b_off(1, R) + e] = sw * (p0 * p2);
    a.ws[b_off(2, R) + e] = sw * (p0 * p1);
    a.ws[c_off(0, R) + e] = sw * (q1 * q2);
    a.ws[c_off(1, R) + e] = sw * (q0 * q2);
    a.ws[c_off(2, R) + e] = sw * (q0 * q1);
    f += sw * ((o0 * o1 * o2 - 2.0 * (q0 * q1 * q2)) + p0 * p1 * p2);
  }
  red[threadIdx.x] = f;
  __syncthreads();
  for (int w = kHistThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && (a.want & kWantLoss)) {
    const T v = a.loss[0] + (T)(0.5 * red[0]);
    a.loss[0] = v;
    if (!isfinite(v)) atomicOr(a.status, (int)kStatusNonFinite);
  }
}

// G_k += grad_scale * (A_k B_k - Abar_k C_k), one output per thread.
template <typename T>
__global__ void __launch_bounds__(kHistThreads) hist_grad(HistArgs<T> a) {
  const int R = a.R;
  const int n0 = a.I[0] * R, n1 = a.I[1] * R, n2 = a.I[2] * R;
  const double sc = a.gscale ? (double)a.gscale[0] : 1.0;
  for (int idx = blockIdx.x * kHistThreads + threadIdx.x; idx < n0 + n1 + n2; idx += gridDim.x * kHistThreads) {
    int k = 0, e = idx;
    if (e >= n0) { e -= n0; k = 1; if (e >= n1) { e -= n1; k = 2; } }
    const int r = e / R, col = e - (e / R) * R;
    const T* Ar = a.A[k] + (size_t)r * R;
    const T* Br = a.Ab[k] + (size_t)r * R;
    const double* B = a.ws + b_off(k, R);
    const double* C = a.ws + c_off(k, R);
    double s = 0.0;
    for (int j = 0; j < R; ++j) s += (double)Ar[j] * B[(size_t)j * R + col] - (double)Br[j] * C[(size_t)j * R + col];
    const T v = a.G[k][e] + (T)(sc * s);
    a.G[k][e] = v;
    if (!isfinite(v)) atomicOr(a.status, (int)kStatusNonFinite);
  }
}

template <typename T>
hipError_t hist_launch(const HistCall& c) {
  HistArgs<T> a;
  for (int k = 0; k < 3; ++k) {
    a.A[k] = static_cast<const T*>(c.A[k]);
    a.Ab[k] = static_cast<const T*>(c.Ab[k]);
    a.G[k] = static_cast<T*>(c.G[k]);
    a.I[k] = c.I[k];
  }
  a.shist = static_cast<const T*>(c.shist);
  a.loss = static_cast<T*>(c.loss);
  a.gscale = static_cast<const T*>(c.grad_scale);
  a.ws = c.ws;
  a.status = c.status;
  a.stamps = c.stamps;
  a.t = c.t;
  a.w = c.w;
  a.theta = c.theta;
  a.R = c.R;
  a.nwin = c.nwin;
  a.want = c.want;
  hipLaunchKernelGGL((hist_gram<T>), dim3(c.R, 9), dim3(kHistThreads), 0, c.stream, a);
  hipLaunchKernelGGL((hist_combine<T>), dim3(1), dim3(kHistThreads), 0, c.stream, a);
  if (c.want & kWantGrad) {
    const int total = (c.I[0] + c.I[1] + c.I[2]) * c.R;
    hipLaunchKernelGGL((hist_grad<T>), dim3((unsigned)std::min(2048, (total + kHistThreads - 1) / kHistThreads)),
                       dim3(kHistThreads), 0, c.stream, a);
  }
  return hipGetLastError();
}

// Gaussian identity: S from s_t and the window, B_k = (*_{l != k} P_l) o S,
// and g_s += 2 (P_0 o P_1 o P_2) s_t (one workgroup).
template <typename T>
__global__ void __launch_bounds__(kHistThreads) id_combine(HistArgs<T> a, const T* st, T* gs) {
  const int R = a.R;
  const double* P = a.ws + gram_off(0, 0, R);
  const size_t RR = (size_t)R * R;
  __shared__ double cw[kMaxWindowModel];
  window_weights(a, cw);
  for (int e = threadIdx.x; e < R * R; e += kHistThreads) {
    const int i = e / R, j = e - (e / R) * R;
    double sw = (double)st[i] * (double)st[j];
    for (int h = 0; h < a.nwin; ++h) sw += cw[h] * (double)a.shist[(size_t)h * R + i] * (double)a.shist[(size_t)h * R + j];
    const double p0 = P[e], p1 = P[RR + e], p2 = P[2 * RR + e];
    a.ws[b_off(0, R) + e] = sw * (p1 * p2);
    a.ws[b_off(1, R) + e] = sw * (p0 * p2);
    a.ws[b_off(2, R) + e] = sw * (p0 * p1);
  }
  for (int i = threadIdx.x; i < R; i += kHistThreads) {
    double s = 0.0;
    for (int j = 0; j < R; ++j) s += P[i * R + j] * P[RR + i * R + j] * P[2 * RR + i * R + j] * (double)st[j];
    const T v = gs[i] + (T)(2.0 * s);
    gs[i] = v;
    if (!isfinite(v)) atomicOr(a.status, (int)kStatusNonFinite);
  }
}

// G_k += 2 A_k B_k, one output per thread.
template <typename T>
__global__ void __launch_bounds__(kHistThreads) id_grad(HistArgs<T> a) {
  const int R = a.R;
  const int n0 = a.I[0] * R, n1 = a.I[1] * R, n2 = a.I[2] * R;
  for (int idx = blockIdx.x * kHistThreads + threadIdx.x; idx < n0 + n1 + n2; idx += gridDim.x * kHistThreads) {
    int k = 0, e = idx;
    if (e >= n0) { e -= n0; k = 1; if (e >= n1) { e -= n1; k = 2; } }
    const int r = e / R, col = e - (e / R) * R;
    const T* Ar = a.A[k] + (size_t)r * R;
    const double* B = a.ws + b_off(k, R);
    double s = 0.0;
    for (int j = 0; j < R; ++j) s += (double)Ar[j] * B[(size_t)j * R + col];
    const T v = a.G[k][e] + (T)(2.0 * s);
    a.G[k][e] = v;
    if (!isfinite(v)) atomicOr(a.status, (int)kStatusNonFinite);
  }
}

template <typename T>
hipError_t ident_launch(const HistCall& c, const void* s_t, void* g_s) {
  HistArgs<T> a;
  for (int k = 0; k < 3; ++k) {
    a.A[k] = static_cast<const T*>(c.A[k]);
    a.Ab[k] = static_cast<const T*>(c.A[k]);
    a.G[k] = static_cast<T*>(c.G[k]);
    a.I[k] = c.I[k];
  }
  a.shist = static_cast<const T*>(c.shist);
  a.loss = nullptr;
  a.gscale = nullptr;
  a.ws = c.ws;
  a.status = c.status;
  a.stamps = c.stamps;
  a.t = c.t;
  a.w = c.w;
  a.theta = c.theta;
  a.R = c.R;
  a.nwin = c.nwin;
  a.want = kWantGrad;
  // Gram matrices A_k'A_k only (the first three of hist_gram's nine)
  hipLaunchKernelGGL((hist_gram<T>), dim3(c.R, 3), dim3(kHistThreads), 0, c.stream, a);
  hipLaunchKernelGGL((id_combine<T>), dim3(1), dim3(kHistThreads), 0, c.stream, a, static_cast<const T*>(s_t),
                     static_cast<T*>(g_s));
  const int total = (c.I[0] + c.I[1] + c.I[2]) * c.R;
  hipLaunchKernelGGL((id_grad<T>), dim3((unsigned)std::min(2048, (total + kHistThreads - 1) / kHistThreads)),
                     dim3(kHistThreads), 0, c.stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t ident_run(const HistCall& c, const void* s_t, void* g_s) {
  return c.dtype == 1 ? ident_launch<double>(c, s_t, g_s) : ident_launch<float>(c, s_t, g_s);
}

namespace {
__global__ void k_set_stamp(int64_t* stamps, int slot, int64_t t) { stamps[slot] = t; }
}  // namespace

hipError_t hist_set_stamp_run(int64_t* stamps, int slot, int64_t t, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_stamp, dim3(1), dim3(1), 0, stream, stamps, slot, t);
  return hipGetLastError();
}

size_t hist_ws_bytes(int R) { return (size_t)15 * R * R * sizeof(double); }

hipError_t hist_run(const HistCall& c) {
  if (c.nwin <= 0 || !(c.want & (kWantLoss | kWantGrad))) return hipSuccess;
  return c.dtype == 1 ? hist_launch<double>(c) : hist_launch<float>(c);
}

}  // namespace gcp
