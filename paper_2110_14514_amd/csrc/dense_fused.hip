// Fused single-pass objective and gradient over a dense slice and its window.
//
// For every entry i of the slice and every slice h of {t} u H_t this computes
// the model m_ih = sum_j s_hj prod_k A^(k)[i_k,j] (eq. CP_model with the
// historical model of eq. gcp_stream_problem_1: stored weight, current
// factors), the loss f and derivative y (Section 2.2), and contracts
//   yhat_ij = sum_h c_h y_ih s_hj
// with the Khatri-Rao rows to give all three factor gradients at once
// (eq. gcp_grad_A per slice, summed with the history weights c_h), plus the
// temporal-weight gradient from the current slice only (eq. gcp_grad_lambda).
// Y, M and the Khatri-Rao matrices are never materialised.
//
// Work decomposition: a workgroup (4 waves) owns a tile of TB1 x TB2 index
// pairs (i1,i2) and all of I3, or, when there are few tiles, one chunk of
// I3 (a second grid dimension).  Lanes run along i3 (coalesced loads of each
// slice row), waves split the tile's pairs.  Per pair, mode-3 contributions
// stay lane-local; the mode-1/2 vector V = sum_i3 yhat * A3[i3] is reduced
// across the wave with a reduce-scatter and added into per-wave LDS rows.
// Partial results of each tile go to a partial buffer that a second kernel
// sums in a fixed order, so results are bitwise reproducible (no atomics).
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kNW = 4;
constexpr int kWG = 64 * kNW;
constexpr int kTBMax = 16;

template <typename T>
struct FusedArgs {
  const T* X[kMaxNs];
  const T* S[kMaxNs];
  T c[kMaxNs];
  const T* A1;
  const T* A2;
  const T* A3;
  T* G1p;
  T* G2p;
  T* G3p;
  T* gsp;
  T* lossp;
  int I1, I2, I3, R, ns, want, tb1, tb2, nb2;
  int nch, cw;  // i3 chunks per tile (blockIdx.y) and their width, a multiple of 64
  size_t rp3;   // row pitch of slices h >= 1 (stored slices); slice 0 has pitch I3
};

struct Tiling {
  int tb1, tb2, nb1, nb2, ntiles, nch, cw;
};

// Few pairs (fewer than 256 tiles of four waves) and long i3 rows: the i3
// range of each tile is split into nch chunks of cw entries, one workgroup
// each, so that about 512 workgroups run.  The chunks of a tile write their
// mode-1 and mode-2 rows, g_s and loss into slots of their own; their G3 rows
// are disjoint.
Tiling tiling_for(int I1, int I2, int I3) {
  long pairs = (long)I1 * I2;
  int tb = pairs >= 200000 ? 16 : (pairs >= 4096 ? 8 : 4);
  Tiling t;
  t.tb1 = t.tb2 = tb;
  t.nb1 = (I1 + tb - 1) / tb;
  t.nb2 = (I2 + tb - 1) / tb;
  t.ntiles = t.nb1 * t.nb2;
  const int c64 = (I3 + 63) / 64;
  int nch = 1;
  if (t.ntiles < 256 && c64 > 1) nch = std::min(c64, (512 + t.ntiles - 1) / t.ntiles);
  t.cw = (c64 + nch - 1) / nch * 64;
  t.nch = I3 > 0 ? (I3 + t.cw - 1) / t.cw : 1;
  return t;
}

struct PartLayout {
  size_t g1, g2, g3, gs, loss, total;
  int s1, s2, s3, s4;           // slots of G1 rows, G2 rows, G3 rows, g_s/loss
};

PartLayout part_layout_slots(int I1, int I2, int I3, int R, size_t es, int s1, int s2, int s3, int s4) {
  PartLayout p;
  p.s1 = s1; p.s2 = s2; p.s3 = s3; p.s4 = s4;
  size_t off = 0;
  p.g1 = off; off = align_up(off + (size_t)s1 * I1 * R * es, 256);
  p.g2 = off; off = align_up(off + (size_t)s2 * I2 * R * es, 256);
  p.g3 = off; off = align_up(off + (size_t)s3 * I3 * R * es, 256);
  p.gs = off; off = align_up(off + (size_t)s4 * R * es, 256);
  p.loss = off; off = align_up(off + (size_t)s4 * es, 256);
  p.total = off;
  return p;
}

PartLayout part_layout(int I1, int I2, int I3, int R, size_t es) {
  Tiling t = tiling_for(I1, I2, I3);
  return part_layout_slots(I1, I2, I3, R, es, t.nb2 * t.nch, t.nb1 * t.nch, t.ntiles, t.ntiles * t.nch);
}

PartLayout part_layout_mfma(int I1, int I2, int I3, int R, int target) {
  MfmaPlan m = mfma_plan(I1, I2, I3, single_tile_waves(R), target, true);
  // mode-1/2 rows per (pair block, I3 chunk), mode-3 rows per tile (the
  // chunks of a tile write disjoint rows), g_s and objective per workgroup
  return part_layout_slots(I1, I2, I3, R, sizeof(float), m.nb2 * m.nch, m.nb1 * m.nch, m.nwg, m.nwg * m.nch);
}

// Reduce-scatter of RT per-lane values over the 64 lanes of a wave.  On
// return the lane holds the wave sum of element jl = lane >> (6 - log2 RT);
// lanes with (lane & (64/RT - 1)) == 0 hold the primary copy.
template <typename T, int RT>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[RT], int lane) {
  int mask = 32;
#pragma unroll
  for (int half = RT / 2; half >= 1; half /= 2) {
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      T send = hi ? v[i] : v[i + half];
      T keep = hi ? v[i + half] : v[i];
      v[i] = keep + __shfl_xor(send, mask);
    }
    mask >>= 1;
  }
  T r = v[0];
  for (; mask >= 1; mask >>= 1) r += __shfl_xor(r, mask);
  return r;
}

template <int RT>
__device__ __forceinline__ int log2c() {
  return RT == 1 ? 0 : RT == 2 ? 1 : RT == 4 ? 2 : RT == 8 ? 3 : RT == 16 ? 4 : RT == 32 ? 5 : 6;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

template <typename T, int LOSS, int RT>
__global__ void __launch_bounds__(kWG) fused_dense_v1(FusedArgs<T> a) {
  __shared__ T a1s[kTBMax][RT];
  __shared__ T a2s[kTBMax][RT];
  __shared__ T g1w[kNW][kTBMax][RT];
  __shared__ T g2w[kNW][kTBMax][RT];
  __shared__ T g3x[64][RT + 1];
  __shared__ T gsx[kNW][RT];
  __shared__ T lsx[kNW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tile = blockIdx.x;
  const int cy = blockIdx.y;
  const int b1 = tile / a.nb2;
  const int b2 = tile % a.nb2;
  const int i10 = b1 * a.tb1;
  const int i20 = b2 * a.tb2;
  const int n1 = min(a.tb1, a.I1 - i10);
  const int n2 = min(a.tb2, a.I2 - i20);
  const int R = a.R;
  const int I2 = a.I2, I3 = a.I3;
  const bool want_loss = a.want & kWantLoss;

  for (int idx = tid; idx < kTBMax * RT; idx += kWG) {
    int r = idx / RT, j = idx % RT;
    a1s[r][j] = (r < n1 && j < R) ? a.A1[(size_t)(i10 + r) * R + j] : T(0);
    a2s[r][j] = (r < n2 && j < R) ? a.A2[(size_t)(i20 + r) * R + j] : T(0);
  }
  for (int idx = tid; idx < kNW * kTBMax * RT; idx += kWG) {
    (&g1w[0][0][0])[idx] = T(0);
    (&g2w[0][0][0])[idx] = T(0);
  }
  __syncthreads();

  T gs[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) gs[j] = T(0);
  Kahan<T> lacc;
  const int npairs = n1 * n2;
  const int jl = lane >> (6 - log2c<RT>());
  const bool primary = (lane & ((64 / RT) - 1)) == 0;

  const int cend = min(I3, (cy + 1) * a.cw);
  for (int c0 = cy * a.cw; c0 < cend; c0 += 64) {
    const int i3 = c0 + lane;
    const bool valid = i3 < I3;
    T a3r[RT], g3[RT];
#pragma unroll
    for (int j = 0; j < RT; ++j) {
      a3r[j] = (valid && j < R) ? a.A3[(size_t)i3 * R + j] : T(0);
      g3[j] = T(0);
    }
    for (int q = wave; q < npairs; q += kNW) {
      const int i1l = q / n2, i2l = q % n2;
      T W[RT], P[RT], yh[RT];
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        W[j] = a1s[i1l][j] * a2s[i2l][j];
        P[j] = W[j] * a3r[j];
        yh[j] = T(0);
      }
      const size_t pr = (size_t)(i10 + i1l) * I2 + (i20 + i2l);
      const size_t off0 = pr * I3 + (valid ? i3 : 0), offr = pr * a.rp3 + (valid ? i3 : 0);
      // the slice values of kPre slices are loaded before any is used, so a
      // wave waits on one HBM round trip per kPre slices, not per slice
      constexpr int kPre = 8;
      for (int h0 = 0; h0 < a.ns; h0 += kPre) {
      T xs[kPre];
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        xs[u] = (valid && h0 + u < a.ns) ? a.X[h0 + u][h0 + u == 0 ? off0 : offr] : T(0);
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int h = h0 + u;
        if (h >= a.ns) break;
        const T* Sh = a.S[h];
        T x = xs[u];
        T m = T(0);
        if (LOSS != kGaussianId) {   // the identity path takes m = 0 (y = -2x)
#pragma unroll
          for (int j = 0; j < RT; ++j)
            if (j < R) m += P[j] * Sh[j];
        }
        T f, y;
        LossFn<T, LOSS>::eval(x, m, f, y);
        const T ch = a.c[h];
        if (want_loss && valid) lacc.add(ch * f);
        y = valid ? y * ch : T(0);
#pragma unroll
        for (int j = 0; j < RT; ++j)
          if (j < R) yh[j] += y * Sh[j];
        if (h == 0) {
#pragma unroll
          for (int j = 0; j < RT; ++j) gs[j] += y * P[j];
        }
      }
      }
      T V[RT];
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        g3[j] += yh[j] * W[j];
        V[j] = yh[j] * a3r[j];
      }
      T v = wave_reduce_scatter<T, RT>(V, lane);
      if (primary) {
        g1w[wave][i1l][jl] += v * a2s[i2l][jl];
        g2w[wave][i2l][jl] += v * a1s[i1l][jl];
      }
    }
    // combine the waves' mode-3 partials for this chunk in a fixed order
    for (int w = 0; w < kNW; ++w) {
      if (wave == w) {
#pragma unroll
        for (int j = 0; j < RT; ++j) g3x[lane][j] = (w == 0 ? T(0) : g3x[lane][j]) + g3[j];
      }
      __syncthreads();
    }
    for (int idx = tid; idx < 64 * RT; idx += kWG) {
      int l = idx / RT, j = idx % RT;
      if (c0 + l < I3 && j < R) a.G3p[((size_t)tile * I3 + c0 + l) * R + j] = g3x[l][j];
    }
    __syncthreads();
  }

  // temporal-weight gradient and loss partials
  {
    T v = wave_reduce_scatter<T, RT>(gs, lane);
    if (primary) gsx[wave][jl] = v;
    T ls = wave_sum(lacc.s);
    if (lane == 0) lsx[wave] = ls;
  }
  __syncthreads();
  for (int idx = tid; idx < kTBMax * RT; idx += kWG) {
    int l = idx / RT, j = idx % RT;
    if (j < R) {
      if (l < n1) {
        T s = g1w[0][l][j];
        for (int w = 1; w < kNW; ++w) s += g1w[w][l][j];
        a.G1p[((size_t)(b2 * a.nch + cy) * a.I1 + i10 + l) * R + j] = s;
      }
      if (l < n2) {
        T s = g2w[0][l][j];
        for (int w = 1; w < kNW; ++w) s += g2w[w][l][j];
        a.G2p[((size_t)(b1 * a.nch + cy) * I2 + i20 + l) * R + j] = s;
      }
    }
  }
  if (tid < R) {
    T s = gsx[0][tid];
    for (int w = 1; w < kNW; ++w) s += gsx[w][tid];
    a.gsp[((size_t)tile * a.nch + cy) * R + tid] = s;
  }
  if (tid == 0) {
    T s = lsx[0];
    for (int w = 1; w < kNW; ++w) s += lsx[w];
    a.lossp[(size_t)tile * a.nch + cy] = s;
  }
}

template <typename T>
struct ReduceArgs {
  const T* G1p;
  const T* G2p;
  const T* G3p;
  const T* gsp;
  const T* lossp;
  const T* A1;
  const T* A2;
  const T* A3;
  const T* st;
  T* G1;
  T* G2;
  T* G3;
  T* gs;
  T* loss;
  T lam, mu;
  T lam3;           // regulariser of the third mode (0 when it is merged modes 3 and 4)
  const T* gscale;
  int I1, I2, I3, R, nb1, nb2, ntiles, nsl, want, gblocks;   // nsl: g_s/loss slots
  int* status;
};

// Sums the partial slots of every output in a fixed order and adds the
// regularisation gradients; the last workgroup forms the objective.  A
// workgroup takes 16 consecutive outputs of one kind (G1, G2, G3 or g_s) and
// splits their slots into 16 fixed chunks: thread (chunk c, output o) sums
// chunk c of output o in slot order (Kahan), with consecutive threads on
// consecutive outputs so that every load is a contiguous row segment; the 16
// chunk sums of an output are then added in chunk order.  Nothing depends
// on scheduling, so results are bitwise reproducible.
template <typename T>
__global__ void __launch_bounds__(256) fused_reduce(ReduceArgs<T> r) {
  const int R = r.R;
  if ((int)blockIdx.x < r.gblocks) {
    __shared__ T part[kRedChunks][kRedOut];
    const int n1 = r.I1 * R, n2 = r.I2 * R, n3 = r.I3 * R;
    const int b1 = (n1 + kRedOut - 1) / kRedOut, b2 = (n2 + kRedOut - 1) / kRedOut;
    const int b3 = (n3 + kRedOut - 1) / kRedOut;
    int blk = blockIdx.x;
    const T* src;
    const T* A;
    size_t stride;
    int slots, nout;
    T* dst;
    T lam = r.lam;
    if (blk < b1) {
      src = r.G1p; stride = n1; slots = r.nb2; nout = n1; A = r.A1; dst = r.G1;
    } else if ((blk -= b1) < b2) {
      src = r.G2p; stride = n2; slots = r.nb1; nout = n2; A = r.A2; dst = r.G2;
    } else if ((blk -= b2) < b3) {
      src = r.G3p; stride = n3; slots = r.ntiles; nout = n3; A = r.A3; dst = r.G3; lam = r.lam3;
    } else {
      blk -= b3;
      src = r.gsp; stride = R; slots = r.nsl; nout = R; A = r.st; dst = r.gs; lam = r.mu;
    }
    const int ol = threadIdx.x % kRedOut, c = threadIdx.x / kRedOut;
    const int o = blk * kRedOut + ol;
    const int s0 = (int)((long)slots * c / kRedChunks), s1 = (int)((long)slots * (c + 1) / kRedChunks);
    Kahan<T> k;
    if (o < nout) kahan_strided(k, src + o, (size_t)s0 * stride, (size_t)s1 * stride, stride, [](T v) { return v; });
    part[c][ol] = k.s;
    __syncthreads();
    if (c == 0 && o < nout) {
      Kahan<T> t;
#pragma unroll
      for (int cc = 0; cc < kRedChunks; ++cc) t.add(part[cc][ol]);
      const T sc = r.gscale ? r.gscale[0] : T(1);
      const T out = sc * (t.s + lam * A[o]);
      dst[o] = out;
      if (!isfinite(out)) atomicOr(r.status, (int)kStatusNonFinite);
    }
    return;
  }
  // objective: data partials + lambda/2 sum ||A||^2 + mu/2 ||s||^2
  __shared__ T red[256];
  const auto id = [](T v) { return v; };
  const auto sq = [](T v) { return v * v; };
  Kahan<T> k;
  kahan_strided(k, r.lossp, threadIdx.x, r.nsl, 256, id);
  Kahan<T> kr;
  kahan_strided(kr, r.A1, threadIdx.x, (size_t)r.I1 * R, 256, sq);
  kahan_strided(kr, r.A2, threadIdx.x, (size_t)r.I2 * R, 256, sq);
  Kahan<T> kr3;   // only used when the third mode has its own regulariser weight
  kahan_strided(r.lam3 == r.lam ? kr : kr3, r.A3, threadIdx.x, (size_t)r.I3 * R, 256, sq);
  Kahan<T> ks;
  kahan_strided(ks, r.st, threadIdx.x, R, 256, sq);
  red[threadIdx.x] = k.s + T(0.5) * r.lam * kr.s + T(0.5) * r.lam3 * kr3.s + T(0.5) * r.mu * ks.s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    r.loss[0] = red[0];
    if (!isfinite(red[0])) atomicOr(r.status, (int)kStatusNonFinite);
  }
}

template <typename T>
hipError_t launch_reduce(const DenseCall& c, const PartLayout& pl) {
  char* base = static_cast<char*>(c.part);
  ReduceArgs<T> r;
  r.G1p = reinterpret_cast<const T*>(base + pl.g1);
  r.G2p = reinterpret_cast<const T*>(base + pl.g2);
  r.G3p = reinterpret_cast<const T*>(base + pl.g3);
  r.gsp = reinterpret_cast<const T*>(base + pl.gs);
  r.lossp = reinterpret_cast<const T*>(base + pl.loss);
  r.A1 = static_cast<const T*>(c.A[0]);
  r.A2 = static_cast<const T*>(c.A[1]);
  r.A3 = static_cast<const T*>(c.A[2]);
  r.st = static_cast<const T*>(c.S[0]);
  r.G1 = static_cast<T*>(c.G[0]);
  r.G2 = static_cast<T*>(c.G[1]);
  r.G3 = static_cast<T*>(c.G[2]);
  r.gs = static_cast<T*>(c.gs);
  r.loss = static_cast<T*>(c.loss_out);
  r.lam = (T)c.lam; r.mu = (T)c.mu;
  r.lam3 = c.merged34 ? T(0) : (T)c.lam;
  r.gscale = static_cast<const T*>(c.grad_scale);
  r.I1 = c.I1; r.I2 = c.I2; r.I3 = c.I3; r.R = c.R;
  r.nb1 = pl.s2; r.nb2 = pl.s1; r.ntiles = pl.s3; r.nsl = pl.s4; r.want = c.want;
  r.status = c.status;
  auto nblk = [](int n) { return (n + kRedOut - 1) / kRedOut; };
  r.gblocks = (c.want & kWantGrad) ? nblk(c.I1 * c.R) + nblk(c.I2 * c.R) + nblk(c.I3 * c.R) + nblk(c.R) : 0;
  const int blocks = r.gblocks + ((c.want & kWantLoss) ? 1 : 0);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((fused_reduce<T>), dim3(blocks), dim3(256), 0, c.stream, r);
  return hipGetLastError();
}

template <typename T, int LOSS, int RT>
hipError_t launch_fused(const DenseCall& c, const Tiling& tl, const PartLayout& pl) {
  FusedArgs<T> a;
  for (int h = 0; h < c.ns; ++h) {
    a.X[h] = static_cast<const T*>(c.X[h]);
    a.S[h] = static_cast<const T*>(c.S[h]);
    a.c[h] = static_cast<T>(c.c[h]);
  }
  char* base = static_cast<char*>(c.part);
  a.A1 = static_cast<const T*>(c.A[0]);
  a.A2 = static_cast<const T*>(c.A[1]);
  a.A3 = static_cast<const T*>(c.A[2]);
  a.G1p = reinterpret_cast<T*>(base + pl.g1);
  a.G2p = reinterpret_cast<T*>(base + pl.g2);
  a.G3p = reinterpret_cast<T*>(base + pl.g3);
  a.gsp = reinterpret_cast<T*>(base + pl.gs);
  a.lossp = reinterpret_cast<T*>(base + pl.loss);
  a.I1 = c.I1; a.I2 = c.I2; a.I3 = c.I3; a.R = c.R; a.ns = c.ns; a.want = c.want;
  a.tb1 = tl.tb1; a.tb2 = tl.tb2; a.nb2 = tl.nb2;
  a.nch = tl.nch; a.cw = tl.cw;
  a.rp3 = c.ring_pitch ? c.ring_pitch : (size_t)c.I3;
  if (c.ev_begin) hipEventRecord(c.ev_begin, c.stream);
  hipLaunchKernelGGL((fused_dense_v1<T, LOSS, RT>), dim3(tl.ntiles, tl.nch), dim3(kWG), 0, c.stream, a);
  hipError_t e = hipGetLastError();
  if (c.ev_end) hipEventRecord(c.ev_end, c.stream);
  if (e != hipSuccess) return e;

  return launch_reduce<T>(c, pl);
}

template <typename T, int LOSS>
hipError_t dispatch_rank(const DenseCall& c, const Tiling& tl, const PartLayout& pl) {
  if (c.R <= 4) return launch_fused<T, LOSS, 4>(c, tl, pl);
  if (c.R <= 8) return launch_fused<T, LOSS, 8>(c, tl, pl);
  if (c.R <= 16) return launch_fused<T, LOSS, 16>(c, tl, pl);
  if (c.R <= 32) return launch_fused<T, LOSS, 32>(c, tl, pl);
  return launch_fused<T, LOSS, 64>(c, tl, pl);
}

template <typename T>
hipError_t dispatch_loss(const DenseCall& c, const Tiling& tl, const PartLayout& pl) {
  switch (c.loss) {
    case kGaussian: return dispatch_rank<T, kGaussian>(c, tl, pl);
    case kPoissonLog: return dispatch_rank<T, kPoissonLog>(c, tl, pl);
    case kBernoulliLogit: return dispatch_rank<T, kBernoulliLogit>(c, tl, pl);
    case kGaussianId: return dispatch_rank<T, kGaussianId>(c, tl, pl);
    case kPoissonId: return dispatch_rank<T, kPoissonId>(c, tl, pl);
    default: return dispatch_rank<T, kBernoulliOdds>(c, tl, pl);
  }
}

}  // namespace

PartLayout part_layout_single(int I1, int I2, int I3, int R) {
  const SsPlan sp = single_slice_plan(I1, I2);
  return part_layout_slots(I1, I2, I3, R, sizeof(float), sp.nb2, sp.nb1, sp.nwg, sp.nwg);
}

size_t dense_fused_part_bytes(int I1, int I2, int I3, int R, int dtype) {
  size_t v = part_layout(I1, I2, I3, R, dtype ? sizeof(double) : sizeof(float)).total;
  if (dtype == 0) {
    for (int i = 0; i < kNumPlanTargets; ++i) v = std::max(v, part_layout_mfma(I1, I2, I3, R, kPlanTargets[i]).total);
    if (R <= 32) v = std::max(v, part_layout_single(I1, I2, I3, R).total);
  }
  return v;
}

hipError_t dense_fused_run(const DenseCall& c) {
  if (single_slice_supported(c)) {
    // one slice: the pairs-in-rows matrix-core kernel
    PartLayout pl = part_layout_single(c.I1, c.I2, c.I3, c.R);
    if (pl.total > c.part_bytes) return hipErrorInvalidValue;
    char* base = static_cast<char*>(c.part);
    if (c.ev_begin) hipEventRecord(c.ev_begin, c.stream);
    hipError_t e = single_slice_launch(c, reinterpret_cast<float*>(base + pl.g1), reinterpret_cast<float*>(base + pl.g2),
                                       reinterpret_cast<float*>(base + pl.g3), reinterpret_cast<float*>(base + pl.gs),
                                       reinterpret_cast<float*>(base + pl.loss));
    if (c.ev_end) hipEventRecord(c.ev_end, c.stream);
    if (e != hipSuccess) return e;
    return launch_reduce<float>(c, pl);
  }
  const bool mfma_ok = mfma_supported(c.R, c.ns, c.dtype);
  bool use_mfma = c.kernel == 2 ? mfma_ok : (c.kernel == 1 ? false : (mfma_ok && c.R > 8));
  // bit-packed slices are read by the matrix-core kernels only
  if (c.xbits) {
    if (!mfma_ok || c.ns > 32 || c.kernel == 1) return hipErrorInvalidValue;
    use_mfma = true;
  }
  if (use_mfma) {
    const int target = c.plan_target > 0 ? c.plan_target : auto_plan_target(c.I1, c.I2, c.I3, c.R, c.ns);
    MfmaPlan mp = mfma_plan(c.I1, c.I2, c.I3, single_tile_waves(c.R), target, true);
    PartLayout pl = part_layout_mfma(c.I1, c.I2, c.I3, c.R, target);
    if (pl.total > c.part_bytes) return hipErrorInvalidValue;
    char* base = static_cast<char*>(c.part);
    if (c.ev_begin) hipEventRecord(c.ev_begin, c.stream);
    hipError_t e = dense_mfma_launch(c, mp, reinterpret_cast<float*>(base + pl.g1),
                                     reinterpret_cast<float*>(base + pl.g2), reinterpret_cast<float*>(base + pl.g3),
                                     reinterpret_cast<float*>(base + pl.gs), reinterpret_cast<float*>(base + pl.loss));
    if (c.ev_end) hipEventRecord(c.ev_end, c.stream);
    if (e != hipSuccess) return e;
    return launch_reduce<float>(c, pl);
  }
  Tiling tl = tiling_for(c.I1, c.I2, c.I3);
  PartLayout pl = part_layout(c.I1, c.I2, c.I3, c.R, c.dtype ? sizeof(double) : sizeof(float));
  if (pl.total > c.part_bytes) return hipErrorInvalidValue;
  return c.dtype ? dispatch_loss<double>(c, tl, pl) : dispatch_loss<float>(c, tl, pl);
}

}  // namespace gcp
