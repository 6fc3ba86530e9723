// Epochs of the factor solver (Algorithm 4) with the ADAM Update of
// Algorithm 2, decided on the device.  The ADAM rate, the iteration index and
// the saved copies (last accepted factors and moments) live in the workspace
// for the whole stream, as the factor ADAM object of Algorithm 1 does; an
// epoch that raised the objective is undone, the rate is multiplied by 0.1 and
// the index goes back tau_f steps.  Every kernel here is tiny or a plain
// streaming copy; the gradients and objectives come from the fused kernels.
#include "solvers.hpp"

namespace gcp {
namespace {

constexpr double kFacDecay = 0.1;

// The bias-corrected rate of the next step (n = i + 1), then i <- i + 1.
__global__ void fac_prep(FacState* st, double beta1, double beta2) {
  if (st->done) return;
  st->p1 *= beta1;
  st->p2 *= beta2;
  st->alpha_t = st->alpha * sqrt(1.0 - st->p2) / (1.0 - st->p1);
  st->i += 1;
}

template <typename T>
__global__ void __launch_bounds__(256) fac_adam(int64_t n, T* __restrict__ a, const T* __restrict__ g,
                                                T* __restrict__ u, T* __restrict__ v, const FacState* st, T b1,
                                                T b2, T eps, T lower) {
  if (st->done) return;
  const T alpha_t = (T)st->alpha_t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const T ge = g[e];
    const T ue = b1 * u[e] + (T(1) - b1) * ge;
    const T ve = b2 * v[e] + (T(1) - b2) * ge * ge;
    u[e] = ue;
    v[e] = ve;
    const T ae = a[e] - alpha_t * ue / (sqrt(ve) + eps);
    a[e] = ae < lower ? lower : ae;
  }
}

// Objective at the start of a solve: F and the stopping test.
template <typename T>
__global__ void fac_begin(FacState* st, const T* loss, double tol) {
  st->F = (double)*loss;
  st->epoch = 0;
  st->rolled = 0ull;
  st->done = !(st->F > tol);
  st->roll = -1;
}

// End of an epoch: keep it, or undo it (the copy kernel moves the data).
template <typename T>
__global__ void fac_decide(FacState* st, const T* loss, int tau, double tol, double beta1, double beta2) {
  if (st->done) {
    st->roll = -1;
    return;
  }
  const double Fv = (double)*loss;
  const int roll = Fv > st->F;
  if (roll) {
    st->alpha *= kFacDecay;
    st->i -= tau;
    st->p1 = pow(beta1, (double)st->i);
    st->p2 = pow(beta2, (double)st->i);
    st->rolled |= 1ull << st->epoch;
  } else {
    st->F = Fv;
  }
  st->epoch += 1;
  st->done = !(st->F > tol);
  st->roll = roll;
}

// roll = 1: A, u, v <- saved copies; roll = 0: saved copies <- A, u, v.
template <typename T>
__global__ void __launch_bounds__(256) fac_copy(int64_t n, T* __restrict__ a, T* __restrict__ u, T* __restrict__ v,
                                                T* __restrict__ ao, T* __restrict__ uo, T* __restrict__ vo,
                                                const FacState* st) {
  const int roll = st->roll;
  if (roll < 0) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (roll) {
      a[e] = ao[e];
      u[e] = uo[e];
      v[e] = vo[e];
    } else {
      ao[e] = a[e];
      uo[e] = u[e];
      vo[e] = v[e];
    }
  }
}

__global__ void fac_init(FacState* st, double alpha) {
  st->F = 0.0;
  st->alpha = alpha;
  st->alpha_t = 0.0;
  st->i = 0;
  st->p1 = 1.0;
  st->p2 = 1.0;
  st->rolled = 0ull;
  st->done = 0;
  st->epoch = 0;
  st->roll = -1;
}

// ---- batched epochs (Algorithm 4 for every stream of a batch) ----
// The same decisions as the single-stream kernels above, one thread (or one
// flattened range of factor entries) per stream; every stream keeps its own
// FacState in its own workspace, so a batch and the stream's own calls share
// the solver state.

__global__ void batch_fac_begin(const BatchDesc* __restrict__ desc, int nstreams) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nstreams) return;
  const BatchDesc& d = desc[i];
  FacState* st = d.fac;
  st->F = (double)d.outloss[0];
  st->epoch = 0;
  st->rolled = 0ull;
  st->done = !(st->F > d.tol_f);
  st->roll = -1;
}

__global__ void batch_fac_prep(const BatchDesc* __restrict__ desc, int nstreams) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nstreams) return;
  FacState* st = desc[i].fac;
  if (st->done) return;
  st->p1 *= desc[i].beta1d;
  st->p2 *= desc[i].beta2d;
  st->alpha_t = st->alpha * sqrt(1.0 - st->p2) / (1.0 - st->p1);
  st->i += 1;
}

// stream of flattened entry o: the last start <= o
__device__ __forceinline__ int stream_of(const int64_t* __restrict__ start, int nstreams, int64_t o) {
  int lo = 0, hi = nstreams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= o) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) batch_fac_adam(const BatchDesc* __restrict__ desc, int nstreams,
                                                      const int64_t* __restrict__ facstart, int64_t nfac) {
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < nfac; o += (int64_t)gridDim.x * 256) {
    const int si = stream_of(facstart, nstreams, o);
    const BatchDesc& d = desc[si];
    const FacState* st = d.fac;
    if (st->done) continue;
    const int64_t e = o - facstart[si];
    const float at = (float)st->alpha_t;
    const float g = d.Gs[e];
    const float u = d.beta1 * d.u[e] + (1.f - d.beta1) * g;
    const float v = d.beta2 * d.v[e] + (1.f - d.beta2) * g * g;
    d.u[e] = u;
    d.v[e] = v;
    const float a = d.A[e] - at * u / (sqrtf(v) + d.eps);
    d.A[e] = a < d.lower ? d.lower : a;
  }
}

__global__ void batch_fac_decide(const BatchDesc* __restrict__ desc, int nstreams, int tau) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nstreams) return;
  const BatchDesc& d = desc[i];
  FacState* st = d.fac;
  if (st->done) {
    st->roll = -1;
    return;
  }
  const double Fv = (double)d.outloss[0];
  const int roll = Fv > st->F;
  if (roll) {
    st->alpha *= kFacDecay;
    st->i -= tau;
    st->p1 = pow(d.beta1d, (double)st->i);
    st->p2 = pow(d.beta2d, (double)st->i);
    st->rolled |= 1ull << st->epoch;
  } else {
    st->F = Fv;
  }
  st->epoch += 1;
  st->done = !(st->F > d.tol_f);
  st->roll = roll;
}

__global__ void __launch_bounds__(256) batch_fac_copy(const BatchDesc* __restrict__ desc, int nstreams,
                                                      const int64_t* __restrict__ facstart, int64_t nfac) {
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < nfac; o += (int64_t)gridDim.x * 256) {
    const int si = stream_of(facstart, nstreams, o);
    const BatchDesc& d = desc[si];
    const int roll = d.fac->roll;
    if (roll < 0) continue;
    const int64_t e = o - facstart[si];
    if (roll) {
      d.A[e] = d.Ao[e];
      d.u[e] = d.uo[e];
      d.v[e] = d.vo[e];
    } else {
      d.Ao[e] = d.A[e];
      d.uo[e] = d.u[e];
      d.vo[e] = d.v[e];
    }
  }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(2048, (n + 255) / 256); }

}  // namespace

hipError_t fac_init_run(FacState* st, double alpha, hipStream_t stream) {
  hipLaunchKernelGGL(fac_init, dim3(1), dim3(1), 0, stream, st, alpha);
  return hipGetLastError();
}

hipError_t fac_step_run(int dtype, int64_t n, void* a, const void* g, void* u, void* v, FacState* st, double beta1,
                        double beta2, double eps, double lower, hipStream_t stream) {
  hipLaunchKernelGGL(fac_prep, dim3(1), dim3(1), 0, stream, st, beta1, beta2);
  if (dtype)
    hipLaunchKernelGGL(fac_adam<double>, dim3(grid_for(n)), dim3(256), 0, stream, n, static_cast<double*>(a),
                       static_cast<const double*>(g), static_cast<double*>(u), static_cast<double*>(v), st, beta1,
                       beta2, eps, lower);
  else
    hipLaunchKernelGGL(fac_adam<float>, dim3(grid_for(n)), dim3(256), 0, stream, n, static_cast<float*>(a),
                       static_cast<const float*>(g), static_cast<float*>(u), static_cast<float*>(v), st,
                       (float)beta1, (float)beta2, (float)eps, lower == -INFINITY ? -INFINITY : (float)lower);
  return hipGetLastError();
}

hipError_t fac_begin_run(int dtype, FacState* st, const void* loss, double tol, hipStream_t stream) {
  if (dtype)
    hipLaunchKernelGGL(fac_begin<double>, dim3(1), dim3(1), 0, stream, st, static_cast<const double*>(loss), tol);
  else
    hipLaunchKernelGGL(fac_begin<float>, dim3(1), dim3(1), 0, stream, st, static_cast<const float*>(loss), tol);
  return hipGetLastError();
}

hipError_t fac_end_epoch_run(int dtype, int64_t n, void* a, void* u, void* v, void* ao, void* uo, void* vo,
                             FacState* st, const void* loss, int tau, double tol, double beta1, double beta2,
                             hipStream_t stream) {
  if (dtype) {
    hipLaunchKernelGGL(fac_decide<double>, dim3(1), dim3(1), 0, stream, st, static_cast<const double*>(loss), tau,
                       tol, beta1, beta2);
    hipLaunchKernelGGL(fac_copy<double>, dim3(grid_for(n)), dim3(256), 0, stream, n, static_cast<double*>(a),
                       static_cast<double*>(u), static_cast<double*>(v), static_cast<double*>(ao),
                       static_cast<double*>(uo), static_cast<double*>(vo), st);
  } else {
    hipLaunchKernelGGL(fac_decide<float>, dim3(1), dim3(1), 0, stream, st, static_cast<const float*>(loss), tau, tol,
                       beta1, beta2);
    hipLaunchKernelGGL(fac_copy<float>, dim3(grid_for(n)), dim3(256), 0, stream, n, static_cast<float*>(a),
                       static_cast<float*>(u), static_cast<float*>(v), static_cast<float*>(ao),
                       static_cast<float*>(uo), static_cast<float*>(vo), st);
  }
  return hipGetLastError();
}

hipError_t batch_fac_begin_run(const BatchRun& b) {
  hipLaunchKernelGGL(batch_fac_begin, dim3((b.nstreams + 63) / 64), dim3(64), 0, b.stream, b.desc, b.nstreams);
  return hipGetLastError();
}

hipError_t batch_fac_step_run(const BatchRun& b) {
  hipLaunchKernelGGL(batch_fac_prep, dim3((b.nstreams + 63) / 64), dim3(64), 0, b.stream, b.desc, b.nstreams);
  hipLaunchKernelGGL(batch_fac_adam, dim3(std::max(1, grid_for(b.nfac))), dim3(256), 0, b.stream, b.desc,
                     b.nstreams, b.facstart, b.nfac);
  return hipGetLastError();
}

hipError_t batch_fac_end_run(const BatchRun& b, int tau_f) {
  hipLaunchKernelGGL(batch_fac_decide, dim3((b.nstreams + 63) / 64), dim3(64), 0, b.stream, b.desc, b.nstreams,
                     tau_f);
  hipLaunchKernelGGL(batch_fac_copy, dim3(std::max(1, grid_for(b.nfac))), dim3(256), 0, b.stream, b.desc,
                     b.nstreams, b.facstart, b.nfac);
  return hipGetLastError();
}

}  // namespace gcp
