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
// Membership of a zero draw is tested in an open-addressing hash table of the
// slice's stored linear indices (capacity a power of two >= 2 nnz, linear
// probing), built when the slice is stored (window slots) or per call (the
// current slice): about one cache line per test, where a binary search over
// the sorted list would fetch a line for most of its log2(nnz) levels.
//
// Work decomposition: a wave takes 64 consecutive draws of one slice.
// Phase 1, one lane per draw: generate the coordinates.  Phase 2, lanes along
// the rank: SEG lanes per draw gather the three factor rows (coalesced row
// reads), form m with a segmented reduction, and add the per-row
// contributions with hardware float atomics; the weight gradient and the
// objective are accumulated in registers and flushed once per wave.
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kMaxAttempts = 64;
constexpr uint64_t kEmptyKey = ~0ull;   // never a linear index (those are < 2^63)

struct SArgs {
  const uint64_t* tab[kMaxNs];     // membership table of slice h
  uint64_t tmask;                  // table capacity - 1
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

// Hash of a linear index into a table of capacity mask + 1 (a power of 2).
__device__ __forceinline__ uint64_t slot_of(uint64_t key, uint64_t mask) {
  return ((key * 0x9E3779B97F4A7C15ull) >> 29) & mask;
}

// Is linear index `key` a stored entry of the slice whose table is `tab`?
__device__ __forceinline__ bool is_stored(const uint64_t* __restrict__ tab, uint64_t mask, uint64_t key) {
  for (uint64_t pos = slot_of(key, mask);; pos = (pos + 1) & mask) {
    const uint64_t v = tab[pos];
    if (v == key) return true;
    if (v == kEmptyKey) return false;
  }
}

// One-pass variant: phase 1 forms one draw per lane; phase 2 takes the
// wave's draws SEG lanes (rank columns) at a time and adds their rows of the
// three MTTKRPs with global atomics.
template <int LOSS, int SEG>
__global__ void __launch_bounds__(256) sampled_kernel(SArgs a) {
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
        ok = !is_stored(a.tab[h], a.tmask, ((uint64_t)i1 * I2 + i2) * I3 + i3);
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
  Kahan<float> lacc;
  const int nd = (int)min<int64_t>(64, total - first);
  const int jc = j < R ? j : 0;
  // U draws per lane group at a time: their lane exchanges and their factor
  // row gathers are all issued before any is used (loads of padded draws and
  // columns read row 0 / column 0 and are masked afterwards, so the loads
  // themselves are unconditional)
  constexpr int U = 4;
  for (int base = 0; base < nd; base += PER * U) {
    int b1[U], b2[U], b3[U];
    float bx[U], bw[U], r1[U], r2[U], r3[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int src = base + PER * u + sub;
      const int sl = src < 64 ? src : 0;
      b1[u] = __shfl(i1, sl);
      b2[u] = __shfl(i2, sl);
      b3[u] = __shfl(i3, sl);
      bx[u] = __shfl(x, sl);
      bw[u] = __shfl(wgt, sl);
      live[u] = src < nd && j < R;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      r1[u] = a.A1[(size_t)b1[u] * R + jc];
      r2[u] = a.A2[(size_t)b2[u] * R + jc];
      r3[u] = a.A3[(size_t)b3[u] * R + jc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float lm = live[u] ? 1.f : 0.f;
      float m = sj * r1[u] * r2[u] * r3[u] * lm;
      for (int o = SEG / 2; o >= 1; o >>= 1) m += __shfl_xor(m, o);
      float f, y;
      LossFn<float, LOSS>::eval(bx[u], m, f, y);
      const float w = base + PER * u + sub < nd ? bw[u] : 0.f;
      const float yt = ch * w * y;
      if (j == 0 && w != 0.f && (a.want & kWantLoss)) lacc.add(ch * w * f);
      if (live[u] && w != 0.f && (a.want & kWantGrad)) {
        const float ys = yt * sj;
        unsafeAtomicAdd(&a.G1[(size_t)b1[u] * R + j], ys * r2[u] * r3[u]);
        unsafeAtomicAdd(&a.G2[(size_t)b2[u] * R + j], ys * r1[u] * r3[u]);
        unsafeAtomicAdd(&a.G3[(size_t)b3[u] * R + j], ys * r1[u] * r2[u]);
        if (cur) gsl += yt * r1[u] * r2[u] * r3[u];
      }
    }
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

// Membership tables: fill with the empty key, then insert every stored
// entry's linear index (compare-and-swap, linear probing; the capacity is at
// least twice the entry count, so a free slot is always found).
__global__ void __launch_bounds__(256) table_fill(uint64_t* __restrict__ tab, uint64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * 256)
    tab[i] = kEmptyKey;
}

__global__ void __launch_bounds__(256) table_insert(const int32_t* __restrict__ coords, int64_t nnz, int I2, int I3,
                                                    unsigned long long* __restrict__ tab, uint64_t mask) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
    const unsigned long long key =
        ((unsigned long long)coords[3 * e] * I2 + (unsigned long long)coords[3 * e + 1]) * I3 + coords[3 * e + 2];
    for (uint64_t pos = slot_of(key, mask);; pos = (pos + 1) & mask) {
      const unsigned long long prev = atomicCAS(&tab[pos], (unsigned long long)kEmptyKey, key);
      if (prev == (unsigned long long)kEmptyKey || prev == key) break;
    }
  }
}

template <int LOSS>
hipError_t launch_seg(const SampledCall& c, const SArgs& a, int64_t blocks) {
  if (c.R <= 16) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 16>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  } else if (c.R <= 32) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 32>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  } else {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 64>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  }
  return hipGetLastError();
}

}  // namespace

uint64_t table_capacity(int64_t max_nnz) {
  uint64_t cap = 64;
  while (cap < 2 * (uint64_t)std::max<int64_t>(max_nnz, 1)) cap <<= 1;
  return cap;
}

hipError_t table_build(const int32_t* coords, int64_t nnz, int I2, int I3, uint64_t* tab, uint64_t cap,
                       hipStream_t stream) {
  const unsigned fb = (unsigned)std::min<uint64_t>(4096, (cap + 255) / 256);
  hipLaunchKernelGGL(table_fill, dim3(fb), dim3(256), 0, stream, tab, cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nnz <= 0) return e;
  const unsigned ib = (unsigned)std::min<int64_t>(8192, (nnz + 255) / 256);
  hipLaunchKernelGGL(table_insert, dim3(ib), dim3(256), 0, stream, coords, nnz, I2, I3,
                     reinterpret_cast<unsigned long long*>(tab), cap - 1);
  return hipGetLastError();
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
    a.tab[h] = c.tab[h];
    a.coords[h] = c.coords[h];
    a.vals[h] = static_cast<const float*>(c.vals[h]);
    a.S[h] = static_cast<const float*>(c.S[h]);
    a.nnz[h] = c.nnz[h];
    a.stamp[h] = (uint32_t)c.stamp[h];
    a.c[h] = (float)c.c[h];
    a.w_nz[h] = c.p > 0 ? (float)((double)c.nnz[h] / (double)c.p) : 0.f;
    a.w_z[h] = c.q > 0 ? (float)((omega - (double)c.nnz[h]) / (double)c.q) : 0.f;
  }
  a.tmask = c.tab_cap - 1;
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
  if (blocks > 0) {
    if (c.ev_begin) (void)hipEventRecord(c.ev_begin, c.stream);
    switch (c.loss) {
      case kGaussian: e = launch_seg<kGaussian>(c, a, blocks); break;
      case kPoissonLog: e = launch_seg<kPoissonLog>(c, a, blocks); break;
      default: e = launch_seg<kBernoulliLogit>(c, a, blocks);
    }
    if (c.ev_end) (void)hipEventRecord(c.ev_end, c.stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sampled_check, dim3(std::min(64, (n1 + n2 + n3 + c.R + 256) / 256)), dim3(256), 0, c.stream,
                     G1, G2, G3, gs, loss, n1, n2, n3, c.R, c.want, c.status);
  return hipGetLastError();
}

}  // namespace gcp
