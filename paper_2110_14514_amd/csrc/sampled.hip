// Stratified sampled objective and gradient on sparse (COO) slices
// (Section 4.3, Algorithm 6).
//
// For every slice h of {t} u H_t, p nonzero draws (uniform over the stored
// entries, with replacement) and q zero draws (uniform index tuples, redrawn
// while they hit a stored entry) each contribute
//   ytilde = c_h * weight * df/dm(x, m),  weight = eta/p or zeta/q,
// to the MTTKRPs of eq. gcp_grad_A (all three modes) and, for the current
// slice, of eq. gcp_grad_lambda; the objective estimate adds
// c_h * weight * f(x, m).  Regularisation terms are exact.
//
// Draws come from Philox4x32-10 (Salmon et al., SC 2011) with key = seed and
// counter = (draw number, slice time stamp, call number, stratum + 2*attempt);
// word k of the output is scaled to [0, n) as floor(word * n / 2^32).
//
// Work decomposition: a wave takes 64 consecutive draws of one slice.
// Phase 1, one lane per draw: generate the coordinates (zero draws test
// membership by binary search over the slice's sorted COO list).  Phase 2,
// lanes along the rank: SEG lanes per draw gather the three factor rows
// (coalesced row reads), form m with a segmented reduction, and add the
// per-row contributions with hardware float atomics; the weight gradient and
// the objective are accumulated in registers and flushed once per wave.
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kMaxAttempts = 64;

struct SArgs {
  const int32_t* coords[kMaxNs];
  const float* vals[kMaxNs];
  const float* S[kMaxNs];
  int64_t nnz[kMaxNs];
  uint32_t stamp[kMaxNs];
  float c[kMaxNs];
  float w_nz[kMaxNs];
  float w_z[kMaxNs];
  const float* A1;
  const float* A2;
  const float* A3;
  float* G1;
  float* G2;
  float* G3;
  float* gs;
  float* loss;
  int* status;
  int I1, I2, I3, R, ns, want;
  int64_t p, q;
  int64_t waves_per_slice;
  uint32_t key0, key1, call;
};

struct Philox {
  uint32_t v[4];
};

__device__ __forceinline__ Philox philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// floor(w * n / 2^32) for n < 2^32
__device__ __forceinline__ int64_t scale_to(uint32_t w, int64_t n) {
  return (int64_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

__device__ __forceinline__ int64_t lin_of(const int32_t* c, int64_t i, int I2, int I3) {
  return ((int64_t)c[3 * i] * I2 + c[3 * i + 1]) * I3 + c[3 * i + 2];
}

// Is linear index `key` a stored entry of the sorted COO list?
__device__ bool is_stored(const int32_t* coords, int64_t nnz, int64_t key, int I2, int I3) {
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t v = lin_of(coords, mid, I2, I3);
    if (v < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < nnz && lin_of(coords, lo, I2, I3) == key;
}

// Draw record of the two-phase variant: the three coordinates and the
// weighted loss derivative c_h * w * y of one draw (zero for a draw that
// contributes nothing).
struct DrawRec {
  int i1, i2, i3;
  float y;
};

// REC = false: one pass; the SEG lanes of a draw add their rank columns of
// the three MTTKRP rows with global atomics.
// REC = true: first phase of the two-phase variant; the draw's record is
// written to recs[h * (p + q) + id] instead, and sampled_scatter forms G.
template <int LOSS, int SEG, bool REC>
__global__ void __launch_bounds__(256) sampled_kernel(SArgs a, DrawRec* __restrict__ recs) {
  const int lane = threadIdx.x & 63;
  const int64_t gwave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int h = (int)(gwave / a.waves_per_slice);
  if (h >= a.ns) return;
  const int64_t first = (gwave - (int64_t)h * a.waves_per_slice) * 64;
  const int64_t total = a.p + a.q;
  const int I1 = a.I1, I2 = a.I2, I3 = a.I3, R = a.R;
  const int32_t* coords = a.coords[h];
  const int64_t nnz = a.nnz[h];

  // phase 1: one draw per lane
  const int64_t id = first + lane;
  int i1 = 0, i2 = 0, i3 = 0;
  float x = 0.f, wgt = 0.f;
  if (id < total && (nnz > 0 || id >= a.p)) {
    if (id < a.p) {
      const Philox r = philox4x32_10((uint32_t)id, a.stamp[h], a.call, 0u, a.key0, a.key1);
      const int64_t e = scale_to(r.v[0], nnz);
      i1 = coords[3 * e];
      i2 = coords[3 * e + 1];
      i3 = coords[3 * e + 2];
      x = a.vals[h][e];
      wgt = a.w_nz[h];
    } else {
      const uint32_t cz = (uint32_t)(id - a.p);  // zero draws may also run with nnz == 0 below
      bool ok = false;
      for (int att = 0; att < kMaxAttempts && !ok; ++att) {
        const Philox r = philox4x32_10(cz, a.stamp[h], a.call, 1u + 2u * (uint32_t)att, a.key0, a.key1);
        i1 = (int)scale_to(r.v[0], I1);
        i2 = (int)scale_to(r.v[1], I2);
        i3 = (int)scale_to(r.v[2], I3);
        ok = !is_stored(coords, nnz, ((int64_t)i1 * I2 + i2) * I3 + i3, I2, I3);
      }
      if (ok) {
        wgt = a.w_z[h];
      } else {
        atomicOr(a.status, (int)kStatusSampler);
        i1 = i2 = i3 = 0;
      }
    }
  }

  // phase 2: SEG lanes per draw, lane = rank column
  constexpr int PER = 64 / SEG;
  const int j = lane % SEG;
  const int sub = lane / SEG;
  const float ch = a.c[h];
  const float sj = j < R ? a.S[h][j] : 0.f;
  const bool cur = h == 0;
  float gsl = 0.f;
  float yown = 0.f;
  Kahan<float> lacc;
  const int nd = (int)min<int64_t>(64, total - first);
  for (int base = 0; base < nd; base += PER) {
    const int src = base + sub;
    const int b1 = __shfl(i1, src), b2 = __shfl(i2, src), b3 = __shfl(i3, src);
    const float bx = __shfl(x, src), bw = __shfl(wgt, src);
    const bool live = src < nd && j < R;
    const float r1 = live ? a.A1[(size_t)b1 * R + j] : 0.f;
    const float r2 = live ? a.A2[(size_t)b2 * R + j] : 0.f;
    const float r3 = live ? a.A3[(size_t)b3 * R + j] : 0.f;
    float m = sj * r1 * r2 * r3;
    for (int o = SEG / 2; o >= 1; o >>= 1) m += __shfl_xor(m, o);
    float f, y;
    LossFn<float, LOSS>::eval(bx, m, f, y);
    const float yt = ch * bw * y;
    if (src < nd && j == 0 && (a.want & kWantLoss)) lacc.add(ch * bw * f);
    if (REC) {
      // hand the draw's derivative back to the lane that owns the draw
      const float yb = __shfl(bw != 0.f ? yt : 0.f, ((lane - base) & (PER - 1)) * SEG);
      if (lane >= base && lane < base + PER) yown = yb;
      if (live && bw != 0.f && cur && (a.want & kWantGrad)) gsl += yt * r1 * r2 * r3;
    } else if (live && bw != 0.f && (a.want & kWantGrad)) {
      const float ys = yt * sj;
      unsafeAtomicAdd(&a.G1[(size_t)b1 * R + j], ys * r2 * r3);
      unsafeAtomicAdd(&a.G2[(size_t)b2 * R + j], ys * r1 * r3);
      unsafeAtomicAdd(&a.G3[(size_t)b3 * R + j], ys * r1 * r2);
      if (cur) gsl += yt * r1 * r2 * r3;
    }
  }
  if (REC && id < total) {
    DrawRec rc;
    rc.i1 = i1;
    rc.i2 = i2;
    rc.i3 = i3;
    rc.y = yown;
    recs[(size_t)h * total + id] = rc;
  }
  if (cur && (a.want & kWantGrad)) {
    for (int o = SEG; o < 64; o <<= 1) gsl += __shfl_xor(gsl, o);
    if (lane < SEG && j < R) unsafeAtomicAdd(&a.gs[j], gsl);
  }
  if (a.want & kWantLoss) {
    float l = lacc.s;
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o);
    if (lane == 0) unsafeAtomicAdd(a.loss, l);
  }
}

// Outputs start from the exact regularisation terms: G = lambda A,
// g_s = mu s_t, loss = lambda/2 sum ||A||^2 + mu/2 ||s_t||^2.
__global__ void __launch_bounds__(256) sampled_init(const float* A1, const float* A2, const float* A3,
                                                    const float* st, float* G1, float* G2, float* G3, float* gs,
                                                    float* loss, int I1, int I2, int I3, int R, float lam, float mu,
                                                    int want) {
  const int n1 = I1 * R, n2 = I2 * R, n3 = I3 * R;
  if ((int)blockIdx.x < (int)gridDim.x - 1) {
    if (!(want & kWantGrad)) return;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n1 + n2 + n3 + R; idx += (gridDim.x - 1) * 256) {
      if (idx < n1)
        G1[idx] = lam * A1[idx];
      else if (idx < n1 + n2)
        G2[idx - n1] = lam * A2[idx - n1];
      else if (idx < n1 + n2 + n3)
        G3[idx - n1 - n2] = lam * A3[idx - n1 - n2];
      else
        gs[idx - n1 - n2 - n3] = mu * st[idx - n1 - n2 - n3];
    }
    return;
  }
  if (!(want & kWantLoss)) return;
  __shared__ float red[256];
  Kahan<float> k;
  const float* mats[3] = {A1, A2, A3};
  const int cnt[3] = {n1, n2, n3};
  for (int m = 0; m < 3; ++m)
    for (int e = threadIdx.x; e < cnt[m]; e += 256) k.add(0.5f * lam * mats[m][e] * mats[m][e]);
  for (int e = threadIdx.x; e < R; e += 256) k.add(0.5f * mu * st[e] * st[e]);
  red[threadIdx.x] = k.s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0];
}

__global__ void sampled_check(const float* G1, const float* G2, const float* G3, const float* gs,
                              const float* loss, int n1, int n2, int n3, int R, int want, int* status) {
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n1 + n2 + n3 + R + 1; idx += gridDim.x * 256) {
    float v;
    if (idx < n1) v = (want & kWantGrad) ? G1[idx] : 0.f;
    else if (idx < n1 + n2) v = (want & kWantGrad) ? G2[idx - n1] : 0.f;
    else if (idx < n1 + n2 + n3) v = (want & kWantGrad) ? G3[idx - n1 - n2] : 0.f;
    else if (idx < n1 + n2 + n3 + R) v = (want & kWantGrad) ? gs[idx - n1 - n2 - n3] : 0.f;
    else v = (want & kWantLoss) ? loss[0] : 0.f;
    if (!isfinite(v)) atomicOr(status, (int)kStatusNonFinite);
  }
}

// Second phase of the two-phase variant.  Workgroup (chunk, k) owns rank
// columns [chunk*RC, chunk*RC + RC) and the k-th of wpc equal runs of the
// draw records; it accumulates its columns of all three MTTKRPs for every
// row in LDS, then adds them to G with one atomic per touched entry.
// kScatterThreads / RC draws are taken per pass, U passes in flight.
constexpr int kScatterThreads = 1024;

template <int RC>
__global__ void __launch_bounds__(kScatterThreads) sampled_scatter(SArgs a, const DrawRec* __restrict__ recs,
                                                                   int64_t ndraws, int wpc) {
  extern __shared__ float acc[];  // (I1 + I2 + I3) x RC
  __shared__ float sS[kMaxNs * RC];
  constexpr int DPI = kScatterThreads / RC;
  constexpr int U = 4;
  const int chunk = blockIdx.x / wpc, k = blockIdx.x - chunk * wpc;
  const int I1 = a.I1, I2 = a.I2, I3 = a.I3, R = a.R;
  const int nrow = I1 + I2 + I3;
  const int c0 = chunk * RC;
  for (int i = threadIdx.x; i < nrow * RC; i += kScatterThreads) acc[i] = 0.f;
  for (int i = threadIdx.x; i < a.ns * RC; i += kScatterThreads) {
    const int h = i / RC, jj = i - h * RC;
    sS[i] = c0 + jj < R ? a.S[h][c0 + jj] : 0.f;
  }
  __syncthreads();
  float* acc1 = acc;
  float* acc2 = acc + I1 * RC;
  float* acc3 = acc + (I1 + I2) * RC;
  const int64_t per = (ndraws + wpc - 1) / wpc;
  const int64_t lo = (int64_t)k * per, hi = min<int64_t>(ndraws, lo + per);
  const int64_t total = a.p + a.q;
  const int jj = threadIdx.x % RC, sub = threadIdx.x / RC;
  const int col = min(c0 + jj, R - 1);
  const bool colok = c0 + jj < R;
  for (int64_t d0 = lo; d0 < hi; d0 += (int64_t)DPI * U) {
    DrawRec rc[U];
    int hh[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t d = d0 + u * DPI + sub;
      if (d < hi) {
        rc[u] = recs[d];
        hh[u] = (int)(d / total);
      } else {
        rc[u].i1 = rc[u].i2 = rc[u].i3 = 0;
        rc[u].y = 0.f;
        hh[u] = 0;
      }
    }
    float v1[U], v2[U], v3[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v1[u] = a.A1[(size_t)rc[u].i1 * R + col];
      v2[u] = a.A2[(size_t)rc[u].i2 * R + col];
      v3[u] = a.A3[(size_t)rc[u].i3 * R + col];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (rc[u].y != 0.f && colok) {
        const float ys = rc[u].y * sS[hh[u] * RC + jj];
        atomicAdd(&acc1[rc[u].i1 * RC + jj], ys * v2[u] * v3[u]);
        atomicAdd(&acc2[rc[u].i2 * RC + jj], ys * v1[u] * v3[u]);
        atomicAdd(&acc3[rc[u].i3 * RC + jj], ys * v1[u] * v2[u]);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nrow * RC; i += kScatterThreads) {
    const int row = i / RC, j = c0 + (i - row * RC);
    const float v = acc[i];
    if (j >= R || v == 0.f) continue;
    if (row < I1)
      unsafeAtomicAdd(&a.G1[(size_t)row * R + j], v);
    else if (row < I1 + I2)
      unsafeAtomicAdd(&a.G2[(size_t)(row - I1) * R + j], v);
    else
      unsafeAtomicAdd(&a.G3[(size_t)(row - I1 - I2) * R + j], v);
  }
}

// LDS available to the accumulators of sampled_scatter (the column chunk of
// S takes the rest).
constexpr size_t kScatterLds = 155648;

// Rank columns per workgroup for the two-phase variant, 0 when even one
// column of the three factors does not fit in LDS.
int scatter_rc(int I1, int I2, int I3, int R) {
  const size_t nrow = (size_t)I1 + I2 + I3;
  int rc = 8;
  while (rc > 1 && (rc / 2 >= R || nrow * rc * 4 > kScatterLds)) rc /= 2;
  return nrow * rc * 4 <= kScatterLds ? rc : 0;
}

template <int LOSS, bool REC>
hipError_t launch_seg(const SampledCall& c, const SArgs& a, int64_t blocks, DrawRec* recs) {
  if (c.R <= 16) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 16, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a, recs);
  } else if (c.R <= 32) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 32, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a, recs);
  } else {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 64, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a, recs);
  }
  return hipGetLastError();
}

template <int LOSS>
hipError_t launch_phase1(const SampledCall& c, const SArgs& a, int64_t blocks, DrawRec* recs) {
  return recs ? launch_seg<LOSS, true>(c, a, blocks, recs) : launch_seg<LOSS, false>(c, a, blocks, nullptr);
}

template <int RC>
hipError_t launch_scatter(const SampledCall& c, const SArgs& a, const DrawRec* recs, int64_t ndraws) {
  const size_t lds = ((size_t)c.I1 + c.I2 + c.I3) * RC * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sampled_scatter<RC>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kScatterLds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  const int nchunk = (c.R + RC - 1) / RC;
  // about one workgroup per compute unit, but no fewer draws per
  // workgroup than accumulator entries it has to clear and flush
  const int64_t rows = (int64_t)c.I1 + c.I2 + c.I3;
  int64_t wpc = std::max<int64_t>(1, (cus + nchunk - 1) / nchunk);
  wpc = std::max<int64_t>(1, std::min<int64_t>(wpc, ndraws / std::max<int64_t>(1, rows)));
  hipLaunchKernelGGL((sampled_scatter<RC>), dim3((unsigned)(nchunk * wpc)), dim3(kScatterThreads), lds, c.stream,
                     a, recs, ndraws, (int)wpc);
  return hipGetLastError();
}

}  // namespace

size_t sampled_scratch_bytes(int I1, int I2, int I3, int R, int ns_max, int64_t p, int64_t q) {
  if (scatter_rc(I1, I2, I3, R) == 0) return 0;
  return (size_t)ns_max * (size_t)(p + q) * sizeof(DrawRec);
}

hipError_t sampled_run(const SampledCall& c) {
  const int n1 = c.I1 * c.R, n2 = c.I2 * c.R, n3 = c.I3 * c.R;
  float* G1 = static_cast<float*>(c.G[0]);
  float* G2 = static_cast<float*>(c.G[1]);
  float* G3 = static_cast<float*>(c.G[2]);
  float* gs = static_cast<float*>(c.gs);
  float* loss = static_cast<float*>(c.loss_out);
  const float* A1 = static_cast<const float*>(c.A[0]);
  const float* A2 = static_cast<const float*>(c.A[1]);
  const float* A3 = static_cast<const float*>(c.A[2]);
  const float* st = static_cast<const float*>(c.S[0]);
  const int gblocks = std::min(1024, (n1 + n2 + n3 + c.R + 255) / 256);
  hipLaunchKernelGGL(sampled_init, dim3(gblocks + 1), dim3(256), 0, c.stream, A1, A2, A3, st, G1, G2, G3, gs,
                     loss, c.I1, c.I2, c.I3, c.R, (float)c.lam, (float)c.mu, c.want);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SArgs a;
  const double omega = (double)c.I1 * c.I2 * c.I3;
  for (int h = 0; h < c.ns; ++h) {
    a.coords[h] = c.coords[h];
    a.vals[h] = static_cast<const float*>(c.vals[h]);
    a.S[h] = static_cast<const float*>(c.S[h]);
    a.nnz[h] = c.nnz[h];
    a.stamp[h] = (uint32_t)c.stamp[h];
    a.c[h] = (float)c.c[h];
    a.w_nz[h] = c.p > 0 ? (float)((double)c.nnz[h] / (double)c.p) : 0.f;
    a.w_z[h] = c.q > 0 ? (float)((omega - (double)c.nnz[h]) / (double)c.q) : 0.f;
  }
  a.A1 = A1; a.A2 = A2; a.A3 = A3;
  a.G1 = G1; a.G2 = G2; a.G3 = G3; a.gs = gs; a.loss = loss;
  a.status = c.status;
  a.I1 = c.I1; a.I2 = c.I2; a.I3 = c.I3; a.R = c.R; a.ns = c.ns; a.want = c.want;
  a.p = c.p; a.q = c.q;
  a.waves_per_slice = (c.p + c.q + 63) / 64;
  a.key0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
  a.key1 = (uint32_t)(c.seed >> 32);
  a.call = (uint32_t)c.call;
  const int64_t blocks = (a.waves_per_slice * c.ns + 3) / 4;
  // two-phase variant when the record buffer was provided and the gradient
  // is wanted; the one-pass kernel otherwise
  const int rc = scatter_rc(c.I1, c.I2, c.I3, c.R);
  const int64_t ndraws = (int64_t)c.ns * (c.p + c.q);
  DrawRec* recs = nullptr;
  if (rc > 0 && (c.want & kWantGrad) && c.rec &&
      c.rec_bytes >= (size_t)ndraws * sizeof(DrawRec))
    recs = static_cast<DrawRec*>(c.rec);
  if (blocks > 0) {
    if (c.ev_begin) (void)hipEventRecord(c.ev_begin, c.stream);
    switch (c.loss) {
      case kGaussian: e = launch_phase1<kGaussian>(c, a, blocks, recs); break;
      case kPoissonLog: e = launch_phase1<kPoissonLog>(c, a, blocks, recs); break;
      default: e = launch_phase1<kBernoulliLogit>(c, a, blocks, recs);
    }
    if (e == hipSuccess && recs) {
      switch (rc) {
        case 8: e = launch_scatter<8>(c, a, recs, ndraws); break;
        case 4: e = launch_scatter<4>(c, a, recs, ndraws); break;
        case 2: e = launch_scatter<2>(c, a, recs, ndraws); break;
        default: e = launch_scatter<1>(c, a, recs, ndraws);
      }
    }
    if (c.ev_end) (void)hipEventRecord(c.ev_end, c.stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sampled_check, dim3(std::min(64, (n1 + n2 + n3 + c.R + 256) / 256)), dim3(256), 0, c.stream,
                     G1, G2, G3, gs, loss, n1, n2, n3, c.R, c.want, c.status);
  return hipGetLastError();
}

}  // namespace gcp
