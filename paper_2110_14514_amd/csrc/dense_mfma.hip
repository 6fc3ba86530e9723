// Matrix-core path: work plan, per-loss dispatch, and the batched path's
// non-tile kernels (reduce, Adam, window).  The tile code is in
// mfma_tile.hpp; its instantiations live in one translation unit per loss
// (dense_mfma_<loss>.hip) so that they compile in parallel.
#include "mfma_tile.hpp"

namespace gcp {

bool mfma_supported(int R, int ns, int dtype) { return dtype == 0 && R >= 1 && R <= 32 && ns <= 64; }

MfmaPlan mfma_plan(int I1, int I2, int I3, int target) {
  (void)I3;
  MfmaPlan p;
  const long pairs = (long)I1 * I2;
  const long target_blocks = target > 0 ? target : kDefaultPlanTarget;
  long per = std::max(1L, (pairs + target_blocks - 1) / target_blocks);
  p.tb2 = (int)std::min<long>(std::min<long>(I2, kTB), per);
  p.tb1 = (int)std::min<long>(std::min<long>(I1, kTB), std::max(1L, per / p.tb2));
  p.nb1 = (I1 + p.tb1 - 1) / p.tb1;
  p.nb2 = (I2 + p.tb2 - 1) / p.tb2;
  p.nblocks = p.nb1 * p.nb2;
  p.nwg = (p.nblocks + kWaves - 1) / kWaves;
  return p;
}

hipError_t dense_mfma_launch(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                             float* gsp, float* lossp) {
  switch (c.loss) {
    case kGaussian: return dense_mfma_launch_gaussian(c, p, G1p, G2p, G3p, gsp, lossp);
    case kPoissonLog: return dense_mfma_launch_poisson(c, p, G1p, G2p, G3p, gsp, lossp);
    default: return dense_mfma_launch_bernoulli(c, p, G1p, G2p, G3p, gsp, lossp);
  }
}

}  // namespace gcp

// ===========================================================================
// Batched path: many independent streams in one persistent launch.
//
// Each stream's per-call state (time index, window fill, slot time stamps,
// Adam iteration) lives in device memory, so a whole time step reads nothing
// from the host and can be captured once as a HIP graph and replayed.  Work
// items (stream, workgroup tile) are listed in decreasing cost; persistent
// workgroups take the next item from a device counter.  Every item writes its
// own partial slots, which the batched reduce sums in a fixed order, so the
// results do not depend on which workgroup ran which item.
// ===========================================================================
namespace gcp {
namespace {

__device__ __forceinline__ uint64_t splitmix64_dev(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float wave_sum_fixed_f(float v) {
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// Outputs of every stream: G1 | G2 | G3 | g_s | loss, one wave per element.
// `outstart` is the prefix sum of per-stream output counts.  The last step
// resets the work counter for the next launch.
__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchDesc* __restrict__ desc, int nstreams,
                                                           const int64_t* __restrict__ outstart, int64_t nout,
                                                           int* __restrict__ counter, int want, int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); o < nout; o += nwaves) {
    int lo = 0, hi = nstreams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (outstart[mid] <= o) lo = mid; else hi = mid - 1;
    }
    const BatchDesc& d = desc[lo];
    const int64_t e = o - outstart[lo];
    const int R = d.R;
    const int n1 = d.I1 * R, n2 = d.I2 * R, n3 = d.I3 * R;
    const float* src;
    int64_t stride;
    int slots;
    float reg;
    float* dst;
    bool is_loss = false;
    if (e < n1) {
      src = d.G1p + e; stride = n1; slots = d.nb2; reg = d.lam * d.A[e]; dst = d.outG[0] + e;
    } else if (e < n1 + n2) {
      const int64_t k = e - n1;
      src = d.G2p + k; stride = n2; slots = d.nb1; reg = d.lam * d.A[d.fac_off1 + k]; dst = d.outG[1] + k;
    } else if (e < n1 + n2 + n3) {
      const int64_t k = e - n1 - n2;
      src = d.G3p + k; stride = n3; slots = d.nwg; reg = d.lam * d.A[d.fac_off2 + k]; dst = d.outG[2] + k;
    } else if (e < n1 + n2 + n3 + R) {
      const int64_t k = e - n1 - n2 - n3;
      src = d.gsp + k; stride = R; slots = d.nwg; reg = d.mu * d.st[k]; dst = d.outgs + k;
    } else {
      is_loss = true;
      src = d.lossp; stride = 1; slots = d.nwg; dst = d.outloss;
      // regularisation of the objective, summed by the same wave
      Kahan<float> kr;
      for (int64_t i = lane; i < d.fac_elems; i += 64) kr.add(d.A[i] * d.A[i]);
      Kahan<float> ks;
      for (int i = lane; i < R; i += 64) ks.add(d.st[i] * d.st[i]);
      reg = 0.5f * d.lam * wave_sum_fixed_f(kr.s) + 0.5f * d.mu * wave_sum_fixed_f(ks.s);
    }
    if (is_loss ? !(want & kWantLoss) : !(want & kWantGrad)) continue;
    Kahan<float> k;
    for (int b = lane; b < slots; b += 64) k.add(src[(int64_t)b * stride]);
    const float sum = wave_sum_fixed_f(k.s);
    if (lane == 0) {
      const float out = sum + reg;
      *dst = out;
      if (!isfinite(out)) atomicOr(status, (int)kStatusNonFinite);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kBatchVariants) counter[threadIdx.x] = 0;
}

// Adam Step (Algorithm 2) over the factor entries of every stream; the
// bias-corrected rate comes from the stream's device-side iteration index.
__global__ void __launch_bounds__(256) batch_adam_kernel(const BatchDesc* __restrict__ desc,
                                                         const BatchState* __restrict__ state, int nstreams,
                                                         const int64_t* __restrict__ facstart, int64_t nfac) {
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < nfac; o += (int64_t)gridDim.x * 256) {
    int lo = 0, hi = nstreams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (facstart[mid] <= o) lo = mid; else hi = mid - 1;
    }
    const BatchDesc& d = desc[lo];
    const int64_t e = o - facstart[lo];
    const double n = (double)(state[lo].adam_i + 1);
    const float at = (float)(d.alpha * sqrt(1.0 - pow(d.beta2d, n)) / (1.0 - pow(d.beta1d, n)));
    const float g = d.Gs[e];
    const float u = d.beta1 * d.u[e] + (1.f - d.beta1) * g;
    const float v = d.beta2 * d.v[e] + (1.f - d.beta2) * g * g;
    d.u[e] = u;
    d.v[e] = v;
    const float a = d.A[e] - at * u / (sqrtf(v) + d.eps);
    d.A[e] = a > d.lower ? a : d.lower;
  }
}

__global__ void batch_adam_tick(BatchState* state, int nstreams) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nstreams) state[i].adam_i += 1;
}

// Reservoir decision of Algorithm 1 for every stream (one thread each):
// append while the window is not full, else j = SplitMix64(seed ^ t) mod t + 1
// replaces slot j-1 when j <= H.  Records the slot for the copy kernel, then
// advances t.
__global__ void batch_window_decide(const BatchDesc* __restrict__ desc, BatchState* __restrict__ state,
                                    int nstreams) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nstreams) return;
  BatchState& s = state[i];
  const int H = desc[i].H;
  int slot = -1;
  if (H > 0) {
    if (s.nwin < H) {
      slot = s.nwin;
      s.nwin += 1;
    } else {
      const uint64_t t = (uint64_t)s.t;
      const uint64_t j = splitmix64_dev(desc[i].seed ^ t) % t + 1;
      if (j <= (uint64_t)H) slot = (int)(j - 1);
    }
  }
  s.pending_slot = slot;
  if (slot >= 0) s.slot_t[slot] = s.t;
  s.t += 1;
}

// Copies X_t and s_t into the chosen window slot and A into A_old.
__global__ void __launch_bounds__(256) batch_window_copy(const BatchDesc* __restrict__ desc,
                                                         const BatchState* __restrict__ state, int nstreams,
                                                         const int64_t* __restrict__ cpystart, int64_t ncpy) {
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < ncpy; o += (int64_t)gridDim.x * 256) {
    int lo = 0, hi = nstreams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cpystart[mid] <= o) lo = mid; else hi = mid - 1;
    }
    const BatchDesc& d = desc[lo];
    const int slot = state[lo].pending_slot;
    int64_t e = o - cpystart[lo];
    if (e < d.fac_elems) {
      d.Aold[e] = d.A[e];
      continue;
    }
    e -= d.fac_elems;
    if (slot < 0) continue;
    if (e < d.omega) {
      // element e of X_t (row pitch I3) to its row of the slot (pitch rp3)
      const int64_t pair = e / d.I3, i3 = e - pair * d.I3;
      d.ring[(int64_t)slot * d.rstride + pair * d.rp3 + i3] = d.Xt[e];
    } else if (e - d.omega < d.R)
      d.shist[(int64_t)slot * d.R + (e - d.omega)] = d.st[e - d.omega];
  }
}

}  // namespace

int batch_variant(int loss, int R, int H, int I3) {
  return loss * 8 + (R > 16 ? 4 : 0) + (H + 1 > 16 ? 2 : 0) + (dma16_ok(I3) ? 1 : 0);
}

bool batch_variant_r16(int v) { return (v & 6) == 0; }

hipError_t batch_grad_run(const BatchRun& b, int want) {
  // one persistent launch per variant present, each over its own slice of
  // the work list
  for (int v = 0; v < kBatchVariants; ++v) {
    if (b.vend[v] <= b.vbegin[v]) continue;
    switch (v >> 3) {
      case 0: batch_launch_gaussian(b, v, want); break;
      case 1: batch_launch_poisson(b, v, want); break;
      default: batch_launch_bernoulli(b, v, want); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int rblocks = (int)std::min<int64_t>(4096, (b.nout + 3) / 4);
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(std::max(1, rblocks)), dim3(256), 0, b.stream, b.desc, b.nstreams,
                     b.outstart, b.nout, b.counter, want, b.status);
  return hipGetLastError();
}

hipError_t batch_adam_run(const BatchRun& b) {
  const int blocks = (int)std::min<int64_t>(2048, (b.nfac + 255) / 256);
  hipLaunchKernelGGL(batch_adam_kernel, dim3(std::max(1, blocks)), dim3(256), 0, b.stream, b.desc, b.state,
                     b.nstreams, b.facstart, b.nfac);
  hipLaunchKernelGGL(batch_adam_tick, dim3((b.nstreams + 63) / 64), dim3(64), 0, b.stream, b.state, b.nstreams);
  return hipGetLastError();
}

hipError_t batch_window_run(const BatchRun& b) {
  hipLaunchKernelGGL(batch_window_decide, dim3((b.nstreams + 63) / 64), dim3(64), 0, b.stream, b.desc, b.state,
                     b.nstreams);
  const int blocks = (int)std::min<int64_t>(8192, (b.ncpy + 255) / 256);
  hipLaunchKernelGGL(batch_window_copy, dim3(std::max(1, blocks)), dim3(256), 0, b.stream, b.desc, b.state,
                     b.nstreams, b.cpystart, b.ncpy);
  return hipGetLastError();
}

}  // namespace gcp
