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
// Work decomposition: a wave takes 4 x 64 consecutive draws of one slice.
// Phase 1, four draws per lane: generate the coordinates, with the random
// reads of the four (COO entry, membership-table slot) issued together.
// Phase 2, lanes along
// the rank: SEG lanes per draw gather the three factor rows (coalesced row
// reads) and form m with a segmented reduction; the weight gradient and the
// objective are accumulated in registers and flushed once per wave.
//
// The MTTKRP rows are then summed in one of two ways.  Row-sorted (default):
// each draw leaves a record (i1, i2, i3, ytilde) and adds one to the count of
// its row in every mode; an exclusive scan of the counts gives each row's
// start; a scatter writes, per mode, the draw's other two indices, its slice
// and ytilde at the next free place of its row; and a segmented reduction
// walks each mode's list in runs of consecutive records, SEG lanes per
// record, keeping the row's sum in registers and adding it to G once per row
// it meets (a handful of atomics per run instead of one per draw and rank
// column).  Atomic: phase 2 adds every draw's three rows to G with hardware
// float atomics (3 R per draw; the L2 atomic rate bounds it).
#include <cstring>

#include "common.hpp"

namespace gcp {
namespace {

constexpr int kMaxAttempts = 64;
constexpr uint64_t kEmptyKey = ~0ull;   // never a linear index (those are < 2^63)

// Record of a draw (row-sorted reduction), at its draw slot gwave * 64 + lane.
struct DrawRec {
  int32_t i1, i2, i3;
  float y;   // ytilde = c_h weight df/dm (0: the draw adds nothing)
};
// Entry of mode k's row-sorted list: the draw's other two indices, its slice
// and ytilde (the row is implied by the position).
struct RowRec {
  int32_t a, b, h;
  float y;
};

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
  DrawRec* rec;                    // row-sorted reduction: draw records
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

// A wave takes kNB x 64 consecutive draws of one slice.  Phase 1 forms kNB
// draws per lane, issuing the random reads of all of them (COO entry or the
// first membership-table slot) before resolving any, so that each wave keeps
// kNB times more of these HBM reads in flight.  Phase 2 takes the draws SEG
// lanes (rank columns) at a time, forms m, f and ytilde, and either adds the
// draw's rows of the three MTTKRPs with global atomics (REC = false) or
// writes the draw's record (REC = true).
constexpr int kNB = 4;

// Phase 1 of a wave's draws of slice h: NB draws per lane, draw number
// first + 64 b + lane for b < NB.  The random reads of all of them (COO
// entry, first membership-table slot) are issued before any is resolved.
// Padded draws (number >= p + q) and nonzero draws of an empty slice get
// weight 0 and index 0; a zero draw that still hits a stored entry after
// kMaxAttempts redraws sets the sampler status and gets weight 0.
template <int NB>
__device__ __forceinline__ void form_draws(const SArgs& a, int h, int64_t first, int lane, int (&i1)[NB],
                                           int (&i2)[NB], int (&i3)[NB], float (&x)[NB], float (&wgt)[NB]) {
  const int64_t total = a.p + a.q;
  const int I1 = a.I1, I2 = a.I2, I3 = a.I3;
  const int32_t* coords = a.coords[h];
  const int64_t nnz = a.nnz[h];
  int64_t e[NB];
  uint64_t key[NB], pos[NB], tv[NB];
  bool nz[NB], zd[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t id = first + 64 * b + lane;
    i1[b] = i2[b] = i3[b] = 0;
    x[b] = 0.f;
    wgt[b] = 0.f;
    nz[b] = id < total && id < a.p && nnz > 0;
    zd[b] = id < total && id >= a.p;
    if (nz[b]) {
      const Philox r = philox4x32_10((uint32_t)id, a.stamp[h], a.call, 0u, a.key0, a.key1);
      e[b] = scale_to(r.v[0], nnz);
    } else {
      e[b] = 0;
    }
    if (zd[b]) {
      const Philox r = philox4x32_10((uint32_t)(id - a.p), a.stamp[h], a.call, 1u, a.key0, a.key1);
      i1[b] = (int)scale_to(r.v[0], I1);
      i2[b] = (int)scale_to(r.v[1], I2);
      i3[b] = (int)scale_to(r.v[2], I3);
      key[b] = ((uint64_t)i1[b] * I2 + i2[b]) * I3 + i3[b];
      pos[b] = slot_of(key[b], a.tmask);
    } else {
      key[b] = 0;
      pos[b] = 0;
    }
  }
  // the random reads of every draw, issued together
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (nz[b]) {
      i1[b] = coords[3 * e[b]];
      i2[b] = coords[3 * e[b] + 1];
      i3[b] = coords[3 * e[b] + 2];
      x[b] = a.vals[h][e[b]];
      wgt[b] = a.w_nz[h];
    }
    tv[b] = zd[b] ? a.tab[h][pos[b]] : 0ull;
  }
  // zero draws: finish the membership test (linear probing), redrawing while
  // the tuple is a stored entry
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!zd[b]) continue;
    const int64_t id = first + 64 * b + lane;
    bool ok = false;
    uint64_t v = tv[b], k = key[b], ps = pos[b];
    for (int att = 0; att < kMaxAttempts;) {
      if (v == kEmptyKey) {
        ok = true;
        break;
      }
      if (v == k) {   // stored: draw again
        if (++att >= kMaxAttempts) break;
        const Philox r = philox4x32_10((uint32_t)(id - a.p), a.stamp[h], a.call, 1u + 2u * (uint32_t)att, a.key0,
                                       a.key1);
        i1[b] = (int)scale_to(r.v[0], I1);
        i2[b] = (int)scale_to(r.v[1], I2);
        i3[b] = (int)scale_to(r.v[2], I3);
        k = ((uint64_t)i1[b] * I2 + i2[b]) * I3 + i3[b];
        ps = slot_of(k, a.tmask);
      } else {
        ps = (ps + 1) & a.tmask;
      }
      v = a.tab[h][ps];
    }
    if (ok) {
      wgt[b] = a.w_z[h];
    } else {
      atomicOr(a.status, (int)kStatusSampler);
      i1[b] = i2[b] = i3[b] = 0;
    }
  }

}


template <int LOSS, int SEG, int CPL, bool REC>
__global__ void __launch_bounds__(256) sampled_kernel(SArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t gwave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int h = (int)(gwave / a.waves_per_slice);
  if (h >= a.ns) return;
  const int64_t first = (gwave - (int64_t)h * a.waves_per_slice) * (64 * kNB);
  const int64_t total = a.p + a.q;
  const int I1 = a.I1, I2 = a.I2, I3 = a.I3, R = a.R;
  const int32_t* coords = a.coords[h];
  const int64_t nnz = a.nnz[h];

  // phase 1: kNB draws per lane (draw first + 64 b + lane)
  int i1[kNB], i2[kNB], i3[kNB];
  float x[kNB], wgt[kNB];
  form_draws<kNB>(a, h, first, lane, i1, i2, i3, x, wgt);

  // phase 2: SEG lanes per draw; lane j holds rank columns j + SEG c, c < CPL
  constexpr int PER = 64 / SEG;
  const int j = lane % SEG;
  const int sub = lane / SEG;
  const float ch = a.c[h];
  float sj[CPL], gsl[CPL];
  int jc[CPL];
  bool jv[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    jv[cc] = j + SEG * cc < R;
    jc[cc] = jv[cc] ? j + SEG * cc : 0;
    sj[cc] = jv[cc] ? a.S[h][jc[cc]] : 0.f;
    gsl[cc] = 0.f;
  }
  const bool cur = h == 0;
  Kahan<float> lacc;
#pragma unroll
  for (int bb = 0; bb < kNB; ++bb) {
    const int64_t fb = first + 64 * bb;
    const int nd = (int)max<int64_t>(0, min<int64_t>(64, total - fb));
    // U draws per lane group at a time: their lane exchanges and their
    // factor row gathers are all issued before any is used (loads of padded
    // draws and columns read row 0 / column 0 and are masked afterwards, so
    // the loads themselves are unconditional)
    constexpr int U = 4;
    for (int base = 0; base < nd; base += PER * U) {
      int b1[U], b2[U], b3[U];
      float bx[U], bw[U], r1[U][CPL], r2[U][CPL], r3[U][CPL];
      bool live[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = base + PER * u + sub;
        const int sl = src < 64 ? src : 0;
        b1[u] = __shfl(i1[bb], sl);
        b2[u] = __shfl(i2[bb], sl);
        b3[u] = __shfl(i3[bb], sl);
        bx[u] = __shfl(x[bb], sl);
        bw[u] = __shfl(wgt[bb], sl);
        live[u] = src < nd;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          r1[u][cc] = a.A1[(size_t)b1[u] * R + jc[cc]];
          r2[u][cc] = a.A2[(size_t)b2[u] * R + jc[cc]];
          r3[u][cc] = a.A3[(size_t)b3[u] * R + jc[cc]];
        }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = base + PER * u + sub;
        const float lm = live[u] ? 1.f : 0.f;
        float m = 0.f;
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) m += sj[cc] * r1[u][cc] * r2[u][cc] * r3[u][cc];
        m *= lm;
        for (int o = SEG / 2; o >= 1; o >>= 1) m += __shfl_xor(m, o);
        float f, y;
        LossFn<float, LOSS>::eval(bx[u], m, f, y);
        const float w = src < nd ? bw[u] : 0.f;
        const float yt = ch * w * y;
        if (j == 0 && w != 0.f && (a.want & kWantLoss)) lacc.add(ch * w * f);
        if constexpr (REC) {
          if (j == 0 && src < nd && (a.want & kWantGrad)) {
            DrawRec rr;
            rr.i1 = b1[u];
            rr.i2 = b2[u];
            rr.i3 = b3[u];
            rr.y = w != 0.f ? yt : 0.f;
            a.rec[(gwave * kNB + bb) * 64 + src] = rr;
          }
          if (live[u] && w != 0.f && (a.want & kWantGrad) && cur)
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) gsl[cc] += yt * r1[u][cc] * r2[u][cc] * r3[u][cc];
        } else {
          if (live[u] && w != 0.f && (a.want & kWantGrad)) {
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) {
              if (!jv[cc]) continue;
              const int jj = jc[cc];
              const float ys = yt * sj[cc];
              unsafeAtomicAdd(&a.G1[(size_t)b1[u] * R + jj], ys * r2[u][cc] * r3[u][cc]);
              unsafeAtomicAdd(&a.G2[(size_t)b2[u] * R + jj], ys * r1[u][cc] * r3[u][cc]);
              unsafeAtomicAdd(&a.G3[(size_t)b3[u] * R + jj], ys * r1[u][cc] * r2[u][cc]);
              if (cur) gsl[cc] += yt * r1[u][cc] * r2[u][cc] * r3[u][cc];
            }
          }
        }
      }
    }
  }
  if (cur && (a.want & kWantGrad)) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      float g = gsl[cc];
      for (int o = SEG; o < 64; o <<= 1) g += __shfl_xor(g, o);
      if (lane < SEG && jv[cc]) unsafeAtomicAdd(&a.gs[jc[cc]], g);
    }
  }
  if (a.want & kWantLoss) {
    float l = lacc.s;
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o);
    if (lane == 0) unsafeAtomicAdd(a.loss, l);
  }
}

// The draws of one slice (SArgs slice 0) as the gradient kernels form them:
// draw number id -> coordinates (3 int32) and weight (eta/p or zeta/q, 0 for
// a zero draw that found no free cell).
__global__ void __launch_bounds__(256) sampled_dump(SArgs a, int32_t* __restrict__ coords_out,
                                                    float* __restrict__ w_out) {
  const int lane = threadIdx.x & 63;
  const int64_t first = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 * kNB);
  const int64_t total = a.p + a.q;
  if (first >= total) return;
  int i1[kNB], i2[kNB], i3[kNB];
  float x[kNB], wgt[kNB];
  form_draws<kNB>(a, 0, first, lane, i1, i2, i3, x, wgt);
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const int64_t id = first + 64 * b + lane;
    if (id < total) {
      coords_out[3 * id] = i1[b];
      coords_out[3 * id + 1] = i2[b];
      coords_out[3 * id + 2] = i3[b];
      w_out[id] = wgt[b];
    }
  }
}

// Row-sorted reduction.  The count and scatter steps take the draw slots in
// chunks of at most kSortChunk per workgroup and keep a histogram of the
// chunk's rows of all three modes in LDS (I1 + I2 + I3 <= kSortBins), so that
// the device sees one atomic per (chunk, row) instead of one per draw.  Small
// draw counts take smaller chunks (down to 1024 slots) so that at least
// kSortMinChunks workgroups run.
constexpr int kSortBins = 12288;
constexpr int kSortChunk = 65536;
constexpr int kSortMinChunks = 512;

int64_t sort_chunk(int64_t nslots) {
  const int64_t want = (nslots + kSortMinChunks - 1) / kSortMinChunks;
  const int64_t c = (want + 1023) / 1024 * 1024;
  return std::min<int64_t>(kSortChunk, std::max<int64_t>(1024, c));
}

__global__ void __launch_bounds__(256) sorted_zero(int* __restrict__ cnt, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) cnt[i] = 0;
}

struct CountArgs {
  const DrawRec* rec;
  int* cnt;             // I1 + I2 + I3 row counts, mode by mode
  int* cur;             // scatter: I1 + I2 + I3 cursors (row starts on entry)
  RowRec* srt[3];       // scatter: the three row-sorted lists
  int64_t slots;        // draw slots per slice (a multiple of 64 kNB)
  int64_t total;        // draws per slice
  int64_t nslots;       // ns * slots
  int64_t chunk;        // slots per workgroup (sort_chunk)
  int I1, I2, I3;
};

// Adds this chunk's valid records (slot inside the slice's draws, nonzero
// ytilde) to the LDS histogram.
__device__ __forceinline__ void chunk_histogram(const CountArgs& a, int* hist, int64_t g0, int64_t g1) {
  const int o2 = a.I1, o3 = a.I1 + a.I2;
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 1024) {
    const int64_t h = g / a.slots;
    if (g - h * a.slots >= a.total) continue;
    const DrawRec r = a.rec[g];
    if (r.y == 0.f) continue;
    atomicAdd(&hist[r.i1], 1);
    atomicAdd(&hist[o2 + r.i2], 1);
    atomicAdd(&hist[o3 + r.i3], 1);
  }
}

// Step 2: row counts.
__global__ void __launch_bounds__(1024) sorted_count(CountArgs a) {
  __shared__ int hist[kSortBins];
  const int nb = a.I1 + a.I2 + a.I3;
  for (int i = threadIdx.x; i < nb; i += 1024) hist[i] = 0;
  __syncthreads();
  const int64_t g0 = (int64_t)blockIdx.x * a.chunk;
  chunk_histogram(a, hist, g0, min(g0 + a.chunk, a.nslots));
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += 1024)
    if (hist[i]) atomicAdd(&a.cnt[i], hist[i]);
}

// Step 4: the chunk's histogram again; one atomic per row reserves the
// chunk's places in that row, and the records are written there (their order
// inside a row is not fixed).
__global__ void __launch_bounds__(1024) sorted_scatter(CountArgs a) {
  __shared__ int hist[kSortBins];
  const int nb = a.I1 + a.I2 + a.I3;
  for (int i = threadIdx.x; i < nb; i += 1024) hist[i] = 0;
  __syncthreads();
  const int64_t g0 = (int64_t)blockIdx.x * a.chunk;
  const int64_t g1 = min(g0 + a.chunk, a.nslots);
  chunk_histogram(a, hist, g0, g1);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += 1024) {
    const int c = hist[i];
    hist[i] = c ? atomicAdd(&a.cur[i], c) : 0;
  }
  __syncthreads();
  const int o2 = a.I1, o3 = a.I1 + a.I2;
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 1024) {
    const int64_t h = g / a.slots;
    if (g - h * a.slots >= a.total) continue;
    const DrawRec r = a.rec[g];
    if (r.y == 0.f) continue;
    RowRec o;
    o.h = (int)h;
    o.y = r.y;
    o.a = r.i2; o.b = r.i3;
    a.srt[0][atomicAdd(&hist[r.i1], 1)] = o;
    o.a = r.i1; o.b = r.i3;
    a.srt[1][atomicAdd(&hist[o2 + r.i2], 1)] = o;
    o.a = r.i1; o.b = r.i2;
    a.srt[2][atomicAdd(&hist[o3 + r.i3], 1)] = o;
  }
}

// Step 3 (after the draw kernel): exclusive scan of each mode's row counts
// into row starts (I_k + 1 values, the last one the list length) and the
// scatter cursors; copy the slices' weight rows into one ns x R table.
struct ScanArgs {
  const int* cnt[3];
  int* start[3];
  int* cur[3];
  int n[3];
  const float* S[kMaxNs];
  float* Sall;
  int ns, R;
};

__global__ void __launch_bounds__(1024) sorted_scan(ScanArgs a) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  for (int k = 0; k < 3; ++k) {
    const int n = a.n[k];
    const int chunk = (n + 1023) / 1024;
    const int t0 = min(n, t * chunk), t1 = min(n, t0 + chunk);
    int s = 0;
    for (int i = t0; i < t1; ++i) s += a.cnt[k][i];
    part[t] = s;
    __syncthreads();
    // inclusive scan of the 1024 chunk sums (Hillis-Steele)
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = part[t] - s;
    for (int i = t0; i < t1; ++i) {
      a.start[k][i] = run;
      a.cur[k][i] = run;
      run += a.cnt[k][i];
    }
    if (t == 1023) a.start[k][n] = part[1023];
    __syncthreads();
  }
  for (int idx = t; idx < a.ns * a.R; idx += 1024) a.Sall[idx] = a.S[idx / a.R][idx % a.R];
}

// Step 5, one launch for the three modes (each block serves one mode, its
// blocks a contiguous range of the grid): a group of SEG lanes (lane j holds rank
// columns j + SEG c, c < CPL) walks a run of consecutive records (reduce_run) of the mode's list, U records at a
// time (their loads and factor-row gathers issued before any is used); the
// row's sum stays in registers and is added to G when the run leaves the row
// and at the end of the run.
constexpr int kRun = 256;

// Run length: kRun, shortened (to no less than 64) when the list is too
// short to give about 8192 runs, but long enough that a row meets about 128
// runs at most: each run ends with R atomics on its last row, and on a mode
// with few rows (24 at rank 50: 0.06 ms for 128 runs per row, 0.08 ms for 300)
// those atomics collide.
int reduce_run(int64_t max_rec, int nrows) {
  auto r8 = [](int64_t v) { return (v + 7) / 8 * 8; };
  const int64_t want = std::max(r8((max_rec + 8191) / 8192), r8(max_rec / (128 * (int64_t)std::max(nrows, 1))));
  return (int)std::min<int64_t>(kRun, std::max<int64_t>(64, want));
}

// The three modes' lists: mode k's blocks are [first[k], first[k + 1]).
struct ReduceModes {
  const RowRec* srt[3];
  const int* start[3];
  const float* Aa[3];
  const float* Ab[3];
  float* G[3];
  int nrows[3], run[3];
  unsigned first[4];
};

template <int SEG, int CPL>
__global__ void __launch_bounds__(256) sorted_reduce(ReduceModes m, const float* __restrict__ Sall, int R) {
  constexpr int PER = 64 / SEG;
  constexpr int U = 8;
  const int k = blockIdx.x < m.first[1] ? 0 : (blockIdx.x < m.first[2] ? 1 : 2);
  const RowRec* __restrict__ srt = m.srt[k];
  const int* __restrict__ start = m.start[k];
  const float* __restrict__ Aa = m.Aa[k];
  const float* __restrict__ Ab = m.Ab[k];
  float* __restrict__ G = m.G[k];
  const int nrows = m.nrows[k], run = m.run[k];
  const unsigned blk = blockIdx.x - m.first[k];
  const int lane = threadIdx.x & 63;
  const int j = lane % SEG, sub = lane / SEG;
  int jc[CPL];
  bool jv[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    jv[cc] = j + SEG * cc < R;
    jc[cc] = jv[cc] ? j + SEG * cc : 0;
  }
  const int64_t grp = ((int64_t)blk * 4 + (threadIdx.x >> 6)) * PER + sub;
  const int64_t nrec = start[nrows];
  const int64_t p0 = grp * run;
  if (p0 >= nrec) return;
  const int64_t p1 = min(p0 + (int64_t)run, nrec);
  // row of p0: the last row whose start is <= p0 (rows may be empty)
  int lo = 0, hi = nrows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= p0) lo = mid; else hi = mid;
  }
  int row = lo;
  int64_t bound = start[row + 1];
  float acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = 0.f;
  auto flush = [&]() {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      if (jv[cc] && acc[cc] != 0.f) unsafeAtomicAdd(&G[(size_t)row * R + jc[cc]], acc[cc]);
      acc[cc] = 0.f;
    }
  };
  for (int64_t pos = p0; pos < p1; pos += U) {
    RowRec r[U];
    float va[U][CPL], vb[U][CPL], vs[U][CPL];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = srt[pos + u < p1 ? pos + u : p0];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        va[u][cc] = Aa[(size_t)r[u].a * R + jc[cc]];
        vb[u][cc] = Ab[(size_t)r[u].b * R + jc[cc]];
        vs[u][cc] = Sall[(size_t)r[u].h * R + jc[cc]];
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (pos + u >= p1) break;
      while (pos + u >= bound) {
        flush();
        ++row;
        bound = start[row + 1];
      }
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] += r[u].y * vs[u][cc] * va[u][cc] * vb[u][cc];
    }
  }
  flush();
}

// Measurement probe for the gather roof of the sampled path: the draw
// kernel's memory pattern with nothing else.  Each wave takes 4 x 64 draws;
// a draw's (i1, i2, i3) come from SplitMix64 of its number (uniform, like the
// Philox draws), SEG lanes gather its three factor rows (four draws' gathers
// issued before any is used), form m = sum_j a1 a2 a3 by a segmented sum, and
// the first lane writes a 16-byte record (i1, i2, i3, m).
__device__ __forceinline__ uint64_t probe_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int SEG, int CPL>
__global__ void __launch_bounds__(256) gather_probe(const float* __restrict__ A1, const float* __restrict__ A2,
                                                    const float* __restrict__ A3, int I1, int I2, int I3, int R,
                                                    int64_t ndraws, uint64_t seed, float4* __restrict__ rec) {
  const int lane = threadIdx.x & 63;
  const int64_t first = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 * kNB);
  int i1[kNB], i2[kNB], i3[kNB];
#pragma unroll
  for (int bb = 0; bb < kNB; ++bb) {
    const uint64_t z = probe_mix(seed ^ (uint64_t)(first + 64 * bb + lane));
    i1[bb] = (int)(((z & 0xFFFFFFFFull) * (uint64_t)I1) >> 32);
    i2[bb] = (int)(((z >> 32) * (uint64_t)I2) >> 32);
    i3[bb] = (int)(((probe_mix(z) & 0xFFFFFFFFull) * (uint64_t)I3) >> 32);
  }
  constexpr int PER = 64 / SEG;
  const int j = lane % SEG, sub = lane / SEG;
  int jc[CPL];
  bool jv[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    jv[cc] = j + SEG * cc < R;
    jc[cc] = jv[cc] ? j + SEG * cc : 0;
  }
#pragma unroll
  for (int bb = 0; bb < kNB; ++bb) {
    const int64_t fb = first + 64 * bb;
    const int nd = (int)max<int64_t>(0, min<int64_t>(64, ndraws - fb));
    constexpr int U = 4;
    for (int base = 0; base < nd; base += PER * U) {
      int b1[U], b2[U], b3[U];
      float r1[U][CPL], r2[U][CPL], r3[U][CPL];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = base + PER * u + sub;
        const int sl = src < 64 ? src : 0;
        b1[u] = __shfl(i1[bb], sl);
        b2[u] = __shfl(i2[bb], sl);
        b3[u] = __shfl(i3[bb], sl);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          r1[u][cc] = A1[(size_t)b1[u] * R + jc[cc]];
          r2[u][cc] = A2[(size_t)b2[u] * R + jc[cc]];
          r3[u][cc] = A3[(size_t)b3[u] * R + jc[cc]];
        }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = base + PER * u + sub;
        float m = 0.f;
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) m += jv[cc] ? r1[u][cc] * r2[u][cc] * r3[u][cc] : 0.f;
        for (int w = SEG / 2; w >= 1; w >>= 1) m += __shfl_xor(m, w);
        if (j == 0 && src < nd)
          rec[fb + src] = make_float4(__int_as_float(b1[u]), __int_as_float(b2[u]), __int_as_float(b3[u]), m);
      }
    }
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
  // eight independent loads in flight per lane before their terms are added
  constexpr int U = 8;
  for (int m = 0; m < 3; ++m)
    for (int e0 = threadIdx.x; e0 < cnt[m]; e0 += 256 * U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = e0 + 256 * u < cnt[m] ? mats[m][e0 + 256 * u] : 0.f;
#pragma unroll
      for (int u = 0; u < U; ++u) k.add(0.5f * lam * v[u] * v[u]);
    }
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

template <int LOSS, bool REC>
hipError_t launch_seg(const SampledCall& c, const SArgs& a, int64_t blocks) {
  // ranks above 32 take two columns per lane, so two draws share a wave
  if (c.R <= 16) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 16, 1, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  } else if (c.R <= 32) {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 32, 1, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  } else {
    hipLaunchKernelGGL((sampled_kernel<LOSS, 32, 2, REC>), dim3((unsigned)blocks), dim3(256), 0, c.stream, a);
  }
  return hipGetLastError();
}

template <bool REC>
hipError_t launch_draws(const SampledCall& c, const SArgs& a, int64_t blocks) {
  switch (c.loss) {
    case kGaussian: return launch_seg<kGaussian, REC>(c, a, blocks);
    case kPoissonLog: return launch_seg<kPoissonLog, REC>(c, a, blocks);
    case kBernoulliLogit: return launch_seg<kBernoulliLogit, REC>(c, a, blocks);
    case kPoissonId: return launch_seg<kPoissonId, REC>(c, a, blocks);
    default: return launch_seg<kBernoulliOdds, REC>(c, a, blocks);
  }
}

// Layout of the row-sorted workspace (byte offsets from its start).
struct SortedLayout {
  size_t rec, srt[3], cnt, S, total;
  int64_t slots;   // draw slots per slice
  size_t cnt_off[3], start_off[3], cur_off[3];   // int offsets inside cnt
};

SortedLayout sorted_layout(int I1, int I2, int I3, int R, int nsmax, int64_t p, int64_t q) {
  SortedLayout L;
  const int64_t total = p + q;
  // a wave's kNB x 64 draw slots per slice, as the draw kernel numbers them
  L.slots = (total + 64 * kNB - 1) / (64 * kNB) * (64 * kNB);
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t off = 0;
  L.rec = off; off = al(off + (size_t)nsmax * L.slots * sizeof(DrawRec));
  for (int k = 0; k < 3; ++k) {
    L.srt[k] = off;
    off = al(off + (size_t)nsmax * total * sizeof(RowRec));
  }
  const int n[3] = {I1, I2, I3};
  size_t io = 0;
  for (int k = 0; k < 3; ++k) { L.cnt_off[k] = io; io += n[k]; }
  for (int k = 0; k < 3; ++k) { L.start_off[k] = io; io += n[k] + 1; }
  for (int k = 0; k < 3; ++k) { L.cur_off[k] = io; io += n[k]; }
  L.cnt = off; off = al(off + io * sizeof(int));
  L.S = off; off = al(off + (size_t)nsmax * R * sizeof(float));
  L.total = off;
  return L;
}

// One launch over the three modes' lists, each at most max_rec records.
template <int SEG, int CPL>
void launch_reduce_modes(const SampledCall& c, ReduceModes m, const float* Sall, int64_t max_rec) {
  unsigned b = 0;
  for (int k = 0; k < 3; ++k) {
    m.run[k] = reduce_run(max_rec, m.nrows[k]);
    const int64_t groups = (max_rec + m.run[k] - 1) / m.run[k];
    m.first[k] = b;
    b += (unsigned)((groups + 4 * (64 / SEG) - 1) / (4 * (64 / SEG)));
  }
  m.first[3] = b;
  if (b > 0)
    hipLaunchKernelGGL((sorted_reduce<SEG, CPL>), dim3(b), dim3(256), 0, c.stream, m, Sall, c.R);
}

}  // namespace

size_t sampled_sorted_bytes(int I1, int I2, int I3, int R, int window, int64_t p, int64_t q) {
  // row counts and starts are 32-bit; the per-chunk row histograms live in LDS
  if ((double)(window + 1) * (double)(p + q) >= 2147483647.0) return 0;
  if ((int64_t)I1 + I2 + I3 > kSortBins) return 0;
  return sorted_layout(I1, I2, I3, R, window + 1, p, q).total;
}

void sampled_sorted_bind(SampledCall& c, char* base, int window) {
  const SortedLayout L = sorted_layout(c.I1, c.I2, c.I3, c.R, window + 1, c.p, c.q);
  c.srec = base + L.rec;
  c.ssrt = base + L.srt[0];
  c.scnt = reinterpret_cast<int*>(base + L.cnt);
  c.sS = reinterpret_cast<float*>(base + L.S);
}

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

hipError_t sampled_dump_run(const SampledCall& c, int h, int32_t* coords, float* weights) {
  if (h < 0 || h >= c.ns) return hipErrorInvalidValue;
  SArgs a;
  memset(&a, 0, sizeof(a));
  const double omega = (double)c.I1 * c.I2 * c.I3;
  a.tab[0] = c.tab[h];
  a.coords[0] = c.coords[h];
  a.vals[0] = static_cast<const float*>(c.vals[h]);
  a.nnz[0] = c.nnz[h];
  a.stamp[0] = (uint32_t)c.stamp[h];
  a.w_nz[0] = c.p > 0 ? (float)((double)c.nnz[h] / (double)c.p) : 0.f;
  a.w_z[0] = c.q > 0 ? (float)((omega - (double)c.nnz[h]) / (double)c.q) : 0.f;
  a.tmask = c.tab_cap - 1;
  a.status = c.status;
  a.I1 = c.I1; a.I2 = c.I2; a.I3 = c.I3; a.R = c.R; a.ns = 1;
  a.p = c.p; a.q = c.q;
  a.key0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
  a.key1 = (uint32_t)(c.seed >> 32);
  a.call = (uint32_t)c.call;
  const int64_t waves = (c.p + c.q + 64 * kNB - 1) / (64 * kNB);
  if (waves == 0) return hipSuccess;
  hipLaunchKernelGGL(sampled_dump, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, c.stream, a, coords, weights);
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
  a.waves_per_slice = (c.p + c.q + 64 * kNB - 1) / (64 * kNB);
  a.key0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
  a.key1 = (uint32_t)(c.seed >> 32);
  a.call = (uint32_t)c.call;
  const int64_t blocks = (a.waves_per_slice * c.ns + 3) / 4;
  const bool sorted = c.srec != nullptr && (c.want & kWantGrad);
  if (blocks > 0) {
    if (c.ev_begin) (void)hipEventRecord(c.ev_begin, c.stream);
    if (!sorted) {
      e = launch_draws<false>(c, a, blocks);
      if (e != hipSuccess) return e;
    } else {
      // the workspace was sized for window + 1 slices; ns <= that
      const SortedLayout L = sorted_layout(c.I1, c.I2, c.I3, c.R, c.ns, c.p, c.q);
      char* base = static_cast<char*>(c.ssrt);
      int* ib = c.scnt;
      const int n[3] = {c.I1, c.I2, c.I3};
      const int ncnt = c.I1 + c.I2 + c.I3;
      hipLaunchKernelGGL(sorted_zero, dim3((unsigned)std::min(1024, (ncnt + 255) / 256)), dim3(256), 0, c.stream,
                         ib, ncnt);
      a.rec = static_cast<DrawRec*>(c.srec);
      e = launch_draws<true>(c, a, blocks);
      if (e != hipSuccess) return e;
      CountArgs ca;
      ca.rec = a.rec;
      ca.cnt = ib + L.cnt_off[0];
      ca.cur = ib + L.cur_off[0];
      RowRec* srt[3];
      for (int k = 0; k < 3; ++k) {
        srt[k] = reinterpret_cast<RowRec*>(base + (L.srt[k] - L.srt[0]));
        ca.srt[k] = srt[k];
      }
      ca.slots = L.slots;
      ca.total = c.p + c.q;
      ca.nslots = (int64_t)c.ns * L.slots;
      ca.I1 = c.I1; ca.I2 = c.I2; ca.I3 = c.I3;
      ca.chunk = sort_chunk(ca.nslots);
      const unsigned nchunks = (unsigned)((ca.nslots + ca.chunk - 1) / ca.chunk);
      hipLaunchKernelGGL(sorted_count, dim3(nchunks), dim3(1024), 0, c.stream, ca);
      ScanArgs sa;
      for (int k = 0; k < 3; ++k) {
        sa.cnt[k] = ib + L.cnt_off[k];
        sa.start[k] = ib + L.start_off[k];
        sa.cur[k] = ib + L.cur_off[k];
        sa.n[k] = n[k];
      }
      for (int h = 0; h < c.ns; ++h) sa.S[h] = static_cast<const float*>(c.S[h]);
      sa.Sall = c.sS;
      sa.ns = c.ns;
      sa.R = c.R;
      hipLaunchKernelGGL(sorted_scan, dim3(1), dim3(1024), 0, c.stream, sa);
      hipLaunchKernelGGL(sorted_scatter, dim3(nchunks), dim3(1024), 0, c.stream, ca);
      // one launch for the three modes; each list holds at most ns (p + q) records
      const int64_t max_rec = (int64_t)c.ns * (c.p + c.q);
      const float* fa[3][2] = {{A2, A3}, {A1, A3}, {A1, A2}};
      float* Gk[3] = {G1, G2, G3};
      ReduceModes m;
      for (int k = 0; k < 3; ++k) {
        m.srt[k] = srt[k];
        m.start[k] = ib + L.start_off[k];
        m.Aa[k] = fa[k][0];
        m.Ab[k] = fa[k][1];
        m.G[k] = Gk[k];
        m.nrows[k] = n[k];
      }
      if (c.R <= 16)
        launch_reduce_modes<16, 1>(c, m, c.sS, max_rec);
      else if (c.R <= 32)
        launch_reduce_modes<32, 1>(c, m, c.sS, max_rec);
      else
        launch_reduce_modes<32, 2>(c, m, c.sS, max_rec);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (c.ev_end) (void)hipEventRecord(c.ev_end, c.stream);
  }
  hipLaunchKernelGGL(sampled_check, dim3(std::min(64, (n1 + n2 + n3 + c.R + 256) / 256)), dim3(256), 0, c.stream,
                     G1, G2, G3, gs, loss, n1, n2, n3, c.R, c.want, c.status);
  return hipGetLastError();
}

hipError_t gather_probe_run(const float* A1, const float* A2, const float* A3, int I1, int I2, int I3, int R,
                            int64_t ndraws, uint64_t seed, void* rec, hipStream_t st) {
  const int64_t waves = (ndraws + 64 * kNB - 1) / (64 * kNB);
  const unsigned blocks = (unsigned)std::max<int64_t>(1, (waves + 3) / 4);
  float4* out = static_cast<float4*>(rec);
  if (R <= 16)
    hipLaunchKernelGGL((gather_probe<16, 1>), dim3(blocks), dim3(256), 0, st, A1, A2, A3, I1, I2, I3, R, ndraws, seed, out);
  else if (R <= 32)
    hipLaunchKernelGGL((gather_probe<32, 1>), dim3(blocks), dim3(256), 0, st, A1, A2, A3, I1, I2, I3, R, ndraws, seed, out);
  else
    hipLaunchKernelGGL((gather_probe<32, 2>), dim3(blocks), dim3(256), 0, st, A1, A2, A3, I1, I2, I3, R, ndraws, seed, out);
  return hipGetLastError();
}

}  // namespace gcp
