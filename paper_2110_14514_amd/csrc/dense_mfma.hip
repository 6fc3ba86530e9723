// Matrix-core path: work plan, per-loss dispatch, and the batched path's
// non-tile kernels (reduce, Adam, window).  The tile code is in
// mfma_tile.hpp; its instantiations live in one translation unit per loss
// (dense_mfma_<loss>.hip) so that they compile in parallel.
#include "mfma_tile.hpp"

namespace gcp {

bool mfma_supported(int R, int ns, int dtype) { return dtype == 0 && R >= 1 && R <= 32 && ns <= 64; }

MfmaPlan mfma_plan(int I1, int I2, int I3, int waves, int target, bool chunk_i3) {
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
  p.nwg = (p.nblocks + waves - 1) / waves;
  // Few pair tiles (a matrix slice of 300 x 300 has 300 pairs): split I3 so
  // that the (tile, chunk) workgroups fill about two per compute unit.
  if (chunk_i3) {
    const int nsc = (I3 + 31) / 32;
    const int slots = 2 * 256;
    if (2 * p.nwg <= slots && nsc > 1) {
      const int want = std::min(nsc, slots / p.nwg);
      p.gpc = (nsc + want - 1) / want;
      p.nch = (nsc + p.gpc - 1) / p.gpc;
    }
  }
  return p;
}

// A launch runs in rounds of resident workgroups (two per compute unit for
// every single-stream build but the rank-16 two-h-tile one, which holds a
// unit alone); a last round of a few workgroups leaves most units idle while
// it runs.  C3 (1000 x 1000 x 64, rank 32): 4096 blocks make 1056 four-wave
// workgroups, 2.06 rounds of 512, and took 3.90 ms; 2048 blocks make 993,
// 1.94 rounds, and took 3.24 ms.  Among 4096, 2048 and 8192 blocks the plan
// with the fullest last round is taken, 4096 unless another fills it
// clearly better.
int auto_plan_target(int I1, int I2, int I3, int R, int ns) {
  static const int cus = [] {
    int d = 0, n = 256;
    if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess)
      n = 256;
    return n;
  }();
  const int per_cu = (R <= 16 && ns > 16) ? 1 : 2;
  const double slots = (double)per_cu * cus;
  int best = kDefaultPlanTarget;
  double best_fill = -1.0;
  for (int t : {kDefaultPlanTarget, 2048, 8192}) {
    const MfmaPlan p = mfma_plan(I1, I2, I3, single_tile_waves(R), t);
    const double rounds = p.nwg / slots;
    const double fill = rounds / std::ceil(rounds);
    if (fill > best_fill + 0.02) {
      best_fill = fill;
      best = t;
    }
  }
  return best;
}

hipError_t dense_mfma_launch(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                             float* gsp, float* lossp) {
  switch (c.loss) {
    case kGaussian: return dense_mfma_launch_gaussian(c, p, G1p, G2p, G3p, gsp, lossp);
    case kPoissonLog: return dense_mfma_launch_poisson(c, p, G1p, G2p, G3p, gsp, lossp);
    case kBernoulliLogit: return dense_mfma_launch_bernoulli(c, p, G1p, G2p, G3p, gsp, lossp);
    case kGaussianId: return dense_mfma_launch_gaussian_id(c, p, G1p, G2p, G3p, gsp, lossp);
    case kPoissonId: return dense_mfma_launch_poisson_id(c, p, G1p, G2p, G3p, gsp, lossp);
    default: return dense_mfma_launch_bernoulli_odds(c, p, G1p, G2p, G3p, gsp, lossp);
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


// Outputs of every stream: G1 | G2 | G3 | g_s | loss; `outstart` is the
// prefix sum of per-stream output counts.  The first nG workgroups take
// kRedOut consecutive gradient outputs each (thread = output column x slot
// chunk, consecutive threads reading consecutive outputs of a slot; the
// chunk sums are added in order), the last nstreams workgroups form the
// objectives.  Nothing depends on scheduling, so the results are bitwise
// reproducible.  The objective workgroup of stream 0 resets the work
// counters for the next launch.
__device__ __forceinline__ int stream_of(const int64_t* __restrict__ outstart, int nstreams, int64_t o) {
  int lo = 0, hi = nstreams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (outstart[mid] <= o) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchDesc* __restrict__ desc, int nstreams,
                                                           const int64_t* __restrict__ outstart, int64_t nout,
                                                           int nG, int* __restrict__ counter, int want,
                                                           int* status) {
  const auto id = [](float v) { return v; };
  if ((int)blockIdx.x < nG) {
    __shared__ float part[kRedChunks][kRedOut];
    const int ol = threadIdx.x % kRedOut, c = threadIdx.x / kRedOut;
    const int64_t o = (int64_t)blockIdx.x * kRedOut + ol;
    bool live = o < nout && (want & kWantGrad);
    const float* src = nullptr;
    const float* A = nullptr;
    float* dst = nullptr;
    int64_t stride = 1, e = 0;
    int slots = 0;
    float lam = 0.f;
    if (live) {
      const BatchDesc& d = desc[stream_of(outstart, nstreams, o)];
      e = o - outstart[stream_of(outstart, nstreams, o)];
      const int R = d.R;
      const int64_t n1 = (int64_t)d.I1 * R, n2 = (int64_t)d.I2 * R, n3 = (int64_t)d.I3 * R;
      lam = d.lam;
      if (e < n1) {
        src = d.G1p; stride = n1; slots = d.nb2; A = d.A; dst = d.outG[0];
      } else if (e < n1 + n2) {
        e -= n1; src = d.G2p; stride = n2; slots = d.nb1; A = d.A + d.fac_off1; dst = d.outG[1];
      } else if (e < n1 + n2 + n3) {
        e -= n1 + n2; src = d.G3p; stride = n3; slots = d.nwg; A = d.A + d.fac_off2; dst = d.outG[2];
      } else if (e < n1 + n2 + n3 + R) {
        e -= n1 + n2 + n3; src = d.gsp; stride = R; slots = d.nwg; A = d.st; dst = d.outgs; lam = d.mu;
      } else {
        live = false;   // the objective: formed by its own workgroup
      }
    }
    Kahan<float> k;
    if (live) {
      const int64_t s0 = (int64_t)slots * c / kRedChunks, s1 = (int64_t)slots * (c + 1) / kRedChunks;
      kahan_strided(k, src + e, (size_t)(s0 * stride), (size_t)(s1 * stride), (size_t)stride, id);
    }
    part[c][ol] = k.s;
    __syncthreads();
    if (c == 0 && live) {
      Kahan<float> t;
#pragma unroll
      for (int cc = 0; cc < kRedChunks; ++cc) t.add(part[cc][ol]);
      const float out = t.s + lam * A[e];
      dst[e] = out;
      if (!isfinite(out)) atomicOr(status, (int)kStatusNonFinite);
    }
    return;
  }
  // objective of stream si: data partials + lambda/2 sum ||A||^2 + mu/2 ||s||^2
  // (the last term left out for the factor solve's objective)
  const int si = (int)blockIdx.x - nG;
  if (si == 0 && threadIdx.x < kBatchVariants) counter[threadIdx.x] = 0;
  if (!(want & kWantLoss)) return;
  const BatchDesc& d = desc[si];
  const auto sq = [](float v) { return v * v; };
  __shared__ float red[256];
  Kahan<float> kl, kr, ks;
  kahan_strided(kl, d.lossp, threadIdx.x, (size_t)d.nwg, 256, id);
  kahan_strided(kr, d.A, threadIdx.x, (size_t)d.fac_elems, 256, sq);
  kahan_strided(ks, d.st, threadIdx.x, (size_t)d.R, 256, sq);
  red[threadIdx.x] = kl.s + 0.5f * d.lam * kr.s + ((want & kWantObjective) ? 0.f : 0.5f * d.mu * ks.s);
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.outloss[0] = red[0];
    if (!isfinite(red[0])) atomicOr(status, (int)kStatusNonFinite);
  }
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
    d.A[e] = a < d.lower ? d.lower : a;
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

int batch_variant(int loss, int R, int H, size_t pitch, int I3) {
  const int mode = H + 1 > 16 ? 1 : (H + 1 <= 8 ? 2 : 0);
  return loss * 12 + (R > 16 ? 6 : 0) + mode * 2 + (copy_mode(pitch, I3) == 2 ? 1 : 0);
}

bool batch_variant_r16(int v) { return v % 12 < 6 && (v % 6) / 2 != 1; }

hipError_t batch_grad_run(const BatchRun& b, int want) {
  // One persistent launch per variant present, each over its own slice of
  // the work list.  The launches are spread over the batch's lanes (HIP
  // streams forked from and joined back into `stream` through events, so a
  // graph capture of `stream` records them as parallel branches): while one
  // variant's workgroups drain at the end of its list, the compute units
  // they free take the next variant's workgroups instead of idling.
  hipError_t e = hipSuccess;
  const int nl = b.nlanes;
  if (nl > 1) {
    e = hipEventRecord(b.fork, b.stream);
    for (int l = 1; l < nl && e == hipSuccess; ++l) e = hipStreamWaitEvent(b.lane[l], b.fork, 0);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < b.nvar; ++i) {
    const int v = b.vorder[i];
    const hipStream_t st = b.vlane[v] == 0 ? b.stream : b.lane[b.vlane[v]];
    switch (v / 12) {
      case 0: batch_launch_gaussian(b, v, want, st); break;
      case 1: batch_launch_poisson(b, v, want, st); break;
      default: batch_launch_bernoulli(b, v, want, st); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int l = 1; l < nl && e == hipSuccess; ++l) {
    e = hipEventRecord(b.join[l], b.lane[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b.stream, b.join[l], 0);
  }
  if (e != hipSuccess) return e;
  const int nG = (int)((b.nout + kRedOut - 1) / kRedOut);
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(nG + b.nstreams), dim3(256), 0, b.stream, b.desc, b.nstreams,
                     b.outstart, b.nout, nG, b.counter, want, b.status);
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
