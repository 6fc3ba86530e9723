// Temporal-weight solver of Algorithm 3 for dense slices: ADAM epochs on s_t
// with the factors held fixed (eq. gcp_stream_temporal_problem), roll-back of
// an epoch that raised the objective with a smaller rate, and the stopping
// test, all decided on the device.  A solve is a fixed sequence of launches
// with no host synchronisation, so it can be captured in a graph.
//
// Over a dense slice the objective and the gradient of the subproblem are
// taken exactly:
//   F(s)    = sum_i f(x_i, m_i) + mu/2 ||s||^2,   m_i = sum_j s_j a1_j a2_j a3_j
//   dF/ds_j = sum_i y_i a1_j a2_j a3_j + mu s_j,   y_i = df/dm(x_i, m_i)
// (the history and factor terms of the step's objective do not depend on s).
//
// One pass over X_t forms either the gradient, followed by the ADAM Step of
// Algorithm 2 on s, or the objective, followed by the epoch decision.  Every
// workgroup of the pass writes a partial sum; a one-workgroup kernel then adds
// the partials in a fixed order and applies the step or the decision, so
// results are bitwise repeatable.  (A last-workgroup ticket in the pass would
// save that launch, but its device-scope fences write back and invalidate the
// L2 of every XCD once per workgroup, which costs far more.)
//
// Work mapping: lane l of a wave owns the mode-3 index i3 = 64 c + l of its
// workgroup's column chunk c and keeps row i3 of A^(3) in registers; a wave
// walks a contiguous run of (i1, i2) rows.  With b_j = a1_j s_j a3_j formed
// when i1 changes, a row costs m = sum_j a2_j b_j and acc2_j += y a2_j
// (2R multiply-adds per entry); acc_j += a1_j acc2_j when i1 changes, and the
// lane's share of the gradient is a3_j acc_j.
#include "solvers.hpp"

namespace gcp {
namespace {

constexpr double kTsDecay = 0.1;   // rate factor of a rolled-back epoch
constexpr int kTsRowUnroll = 4;    // slice rows whose loads are in flight together
constexpr int kTsTargetBlocks = 512;        // workgroups per pass (two per compute unit)

enum TsMode { kTsGrad = 0, kTsObjInit = 1, kTsObjEpoch = 2 };

template <typename T>
struct TsArgs {
  const T* X;
  const T* A1;        // factors copied with rows padded to the rank tile (zeros past R)
  const T* A2;
  const T* A3;
  T* s;               // the weights (caller's output buffer)
  T* u;
  T* v;
  T* so;              // last accepted s, u, v
  T* uo;
  T* vo;
  T* part;            // nblk x (R + 1): gradient partials, then the objective partial
  TsgdState* st;
  int* status;
  int I1, I2, I3, R;
  int nchunk;         // column chunks of 64 mode-3 indices
  int rows_per_grp;   // (i1, i2) rows per workgroup
  int nblk;
  int tau;
  T mu, lower, b1, b2, eps;
  double beta1, beta2, tol;
};

template <typename T, int LOSS>
struct TsLoss {
  __device__ __forceinline__ static void fy(T x, T m, T& f, T& y) { LossFn<T, LOSS>::eval(x, m, f, y); }
};
template <int LOSS>
struct TsLoss<float, LOSS> {
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) { LossFast<LOSS>::fy(x, m, f, y); }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Adds the partial slots of columns col0 .. col0 + ncol - 1 (ncol <= C, C a
// power of 2 dividing NT) over all workgroups in a fixed order: thread
// t = q C + j sums column j over workgroups q, q + NT/C, ..., and a fixed tree
// over q combines the sums.  Returns column j's total in thread j.
template <typename T, int NT, int C>
__device__ T sum_cols(const T* part, int nblk, int stride, int col0, int ncol, T* red) {
  const int j = threadIdx.x % C;
  const int q = threadIdx.x / C;
  Kahan<T> k;
  if (j < ncol)
    kahan_strided(k, part + col0 + j, (size_t)q * stride, (size_t)nblk * stride, (size_t)(NT / C) * stride,
                  [](T v) { return v; });
  red[threadIdx.x] = k.s;
  __syncthreads();
#pragma unroll
  for (int w = NT / C / 2; w >= 1; w >>= 1) {
    if (q < w) red[threadIdx.x] += red[threadIdx.x + w * C];
    __syncthreads();
  }
  return (int)threadIdx.x < C ? red[threadIdx.x] : T(0);
}

// Epoch bookkeeping on the objective Fv (thread 0): at the start F <- Fv;
// after an epoch keep it (F <- Fv) or roll back (rate x decay, index back
// tau, powers recomputed); then the stopping test.  Returns 1 for a roll-back.
template <typename T>
__device__ int ts_decide(const TsArgs<T>& a, T Fv, bool init) {
  TsgdState* st = a.st;
  if (!isfinite(Fv)) atomicOr(a.status, (int)kStatusNonFinite);
  int roll = 0;
  if (init) {
    st->F = (double)Fv;
  } else {
    roll = (double)Fv > st->F;
    if (roll) {
      st->alpha *= kTsDecay;
      st->i -= a.tau;
      st->p1 = pow(a.beta1, (double)st->i);
      st->p2 = pow(a.beta2, (double)st->i);
      st->rolled |= 1ull << st->epoch;
    } else {
      st->F = (double)Fv;
    }
    st->epoch += 1;
  }
  st->done = !(st->F > a.tol);
  return roll;
}

// ADAM Update: s, u, v back to the saved copies, or the copies refreshed
// (threads j < R; s_now holds s as the epoch left it).
template <typename T>
__device__ void ts_keep_or_undo(const TsArgs<T>& a, int roll, const T* s_now) {
  const int j = threadIdx.x;
  if (j >= a.R) return;
  if (roll) {
    a.s[j] = a.so[j];
    a.u[j] = a.uo[j];
    a.v[j] = a.vo[j];
  } else {
    a.so[j] = s_now[j];
    a.uo[j] = a.u[j];
    a.vo[j] = a.v[j];
  }
}

template <typename T, int LOSS, int RK, int MODE, int NT>
__global__ void __launch_bounds__(NT) ts_pass(TsArgs<T> a) {
  constexpr int W = NT / 64;
  constexpr bool GRAD = MODE == kTsGrad;
  __shared__ T sh_s[RK];
  __shared__ T sh_w[W][RK + 1];
  // written only by earlier launches, so every workgroup reads the same value
  if (a.st->done) return;

  const int R = a.R;
  const int lane = threadIdx.x & 63;
  // wave-uniform: the factor rows a wave reads come through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if ((int)threadIdx.x < RK) sh_s[threadIdx.x] = (int)threadIdx.x < R ? a.s[threadIdx.x] : T(0);
  __syncthreads();

  const int chunk = blockIdx.x % a.nchunk;
  const int grp = blockIdx.x / a.nchunk;
  const int i3 = chunk * 64 + lane;
  const bool valid = i3 < a.I3;
  // row i3 of A^(3) is read where it is used (at each change of i1 and at
  // the end), which keeps it out of the registers of the row loop
  const T* a3p = a.A3 + (size_t)(valid ? i3 : 0) * RK;
  const T vmask = valid ? T(1) : T(0);

  // rows of this wave: a contiguous run of (i1, i2); I1 I2 < 2^31
  const int nrows = a.I1 * a.I2;
  const int g0 = grp * a.rows_per_grp;
  const int g1 = min(g0 + a.rows_per_grp, nrows);
  const int per_wave = (g1 - g0 + W - 1) / W;
  const int r0 = min(g0 + wave * per_wave, g1);
  const int r1 = min(r0 + per_wave, g1);

  T b[RK], acc[RK], acc2[RK];
#pragma unroll
  for (int j = 0; j < RK; ++j) acc[j] = acc2[j] = b[j] = T(0);
  T lacc = T(0);
  // b_j = a1_j s_j a3_j for mode-1 index i1
  auto load_b = [&](int i1) {
#pragma unroll
    for (int j = 0; j < RK; ++j) b[j] = a.A1[(size_t)i1 * RK + j] * sh_s[j] * (vmask * a3p[j]);
  };
  // acc_j += a1_j acc2_j for the rows of mode-1 index i1 just finished
  auto flush = [&](int i1) {
#pragma unroll
    for (int j = 0; j < RK; ++j) {
      acc[j] += a.A1[(size_t)i1 * RK + j] * acc2[j];
      acc2[j] = T(0);
    }
  };

  if (r0 < r1) {
    int i1 = r0 / a.I2;
    int i2 = r0 - i1 * a.I2;
    load_b(i1);
    // lanes past I3 read a valid duplicate entry; their terms are masked
    const int i3c = valid ? i3 : a.I3 - 1;
    const int last = r1 - 1;
    T xn[kTsRowUnroll];
#pragma unroll
    for (int u = 0; u < kTsRowUnroll; ++u) xn[u] = a.X[(size_t)min(r0 + u, last) * a.I3 + i3c];
    T a2n[RK];
#pragma unroll
    for (int j = 0; j < RK; ++j) a2n[j] = a.A2[(size_t)i2 * RK + j];
    for (int r = r0; r < r1; r += kTsRowUnroll) {
      T x[kTsRowUnroll];
#pragma unroll
      for (int u = 0; u < kTsRowUnroll; ++u) {
        x[u] = xn[u];
        // next rows' loads are in flight while these rows are processed
        xn[u] = a.X[(size_t)min(r + kTsRowUnroll + u, last) * a.I3 + i3c];
      }
#pragma unroll
      for (int u = 0; u < kTsRowUnroll; ++u) {
        if (r + u >= r1) break;
        T a2[RK];
        // the next row's a2 is requested before this row's arithmetic
        const int i2n = i2 + 1 == a.I2 ? 0 : i2 + 1;
#pragma unroll
        for (int j = 0; j < RK; ++j) {
          a2[j] = a2n[j];
          a2n[j] = a.A2[(size_t)i2n * RK + j];
        }
        T m0 = T(0), m1 = T(0);
#pragma unroll
        for (int j = 0; j < RK; j += 2) {
          m0 += a2[j] * b[j];
          m1 += a2[j + 1] * b[j + 1];
        }
        T f, y;
        TsLoss<T, LOSS>::fy(x[u], m0 + m1, f, y);
        if (GRAD) {
#pragma unroll
          for (int j = 0; j < RK; ++j) acc2[j] += y * a2[j];
        } else {
          lacc += valid ? f : T(0);
        }
        if (++i2 == a.I2) {
          if (GRAD) flush(i1);
          i2 = 0;
          ++i1;
          if (r + u + 1 < r1) load_b(i1);
        }
      }
    }
    if (GRAD && i2 != 0) flush(i1);
  }

  T* prow = a.part + (size_t)blockIdx.x * (R + 1);
  if (GRAD) {
    // lanes past I3 hold a3 = 0 and contribute nothing
#pragma unroll
    for (int j = 0; j < RK; ++j) {
      const T pj = wave_sum(vmask * a3p[j] * acc[j]);
      if (lane == 0) sh_w[wave][j] = pj;
    }
    __syncthreads();
    if ((int)threadIdx.x < R) {
      T t = T(0);
#pragma unroll
      for (int w = 0; w < W; ++w) t += sh_w[w][threadIdx.x];
      prow[threadIdx.x] = t;
    }
  } else {
    const T pl = wave_sum(lacc);
    if (lane == 0) sh_w[wave][RK] = pl;
    __syncthreads();
    if (threadIdx.x == 0) {
      T t = T(0);
#pragma unroll
      for (int w = 0; w < W; ++w) t += sh_w[w][RK];
      prow[R] = t;
    }
  }

}

// One workgroup: adds the pass's partial slots in a fixed order, then the
// ADAM Step on s (gradient pass) or the epoch decision (objective pass).
template <typename T, int RK, int MODE, int NT>
__global__ void __launch_bounds__(NT) ts_final(TsArgs<T> a) {
  __shared__ T sh_s[RK];
  __shared__ T sh_red[NT];
  __shared__ int sh_roll;
  TsgdState* st = a.st;
  if (st->done) return;
  const int R = a.R;
  if ((int)threadIdx.x < RK) sh_s[threadIdx.x] = (int)threadIdx.x < R ? a.s[threadIdx.x] : T(0);
  __syncthreads();
  if (MODE == kTsGrad) {
    T gj = sum_cols<T, NT, RK>(a.part, a.nblk, R + 1, 0, R, sh_red);
    if ((int)threadIdx.x < R) {
      const int j = threadIdx.x;
      gj += a.mu * sh_s[j];
      if (!isfinite(gj)) atomicOr(a.status, (int)kStatusNonFinite);
      // bias correction with n = i + 1 from the carried powers beta^i
      const double p1 = st->p1 * a.beta1, p2 = st->p2 * a.beta2;
      const T alpha_t = (T)(st->alpha * sqrt(1.0 - p2) / (1.0 - p1));
      const T uj = a.b1 * a.u[j] + (T(1) - a.b1) * gj;
      const T vj = a.b2 * a.v[j] + (T(1) - a.b2) * gj * gj;
      a.u[j] = uj;
      a.v[j] = vj;
      const T sj = sh_s[j] - alpha_t * uj / (sqrt(vj) + a.eps);
      a.s[j] = sj < a.lower ? a.lower : sj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      st->i += 1;
      st->p1 *= a.beta1;
      st->p2 *= a.beta2;
    }
    return;
  }

  const T data = sum_cols<T, NT, 1>(a.part, a.nblk, R + 1, R, 1, sh_red);
  if (threadIdx.x == 0) {
    T reg = T(0);
    for (int j = 0; j < R; ++j) reg += sh_s[j] * sh_s[j];
    sh_roll = ts_decide(a, data + T(0.5) * a.mu * reg, MODE == kTsObjInit);
  }
  __syncthreads();
  if (MODE == kTsObjEpoch) ts_keep_or_undo(a, sh_roll, sh_s);
}

// Sampled (COO) variant: the ADAM Step on s from a weight gradient g (which
// holds mu s already), then i <- i + 1.  One workgroup of 64 threads.
template <typename T>
__global__ void ts_step_from(TsArgs<T> a, const T* g) {
  TsgdState* st = a.st;
  if (st->done) return;
  const int j = threadIdx.x;
  if (j < a.R) {
    const double p1 = st->p1 * a.beta1, p2 = st->p2 * a.beta2;
    const T alpha_t = (T)(st->alpha * sqrt(1.0 - p2) / (1.0 - p1));
    const T gj = g[j];
    if (!isfinite(gj)) atomicOr(a.status, (int)kStatusNonFinite);
    const T uj = a.b1 * a.u[j] + (T(1) - a.b1) * gj;
    const T vj = a.b2 * a.v[j] + (T(1) - a.b2) * gj * gj;
    a.u[j] = uj;
    a.v[j] = vj;
    const T sj = a.s[j] - alpha_t * uj / (sqrt(vj) + a.eps);
    a.s[j] = sj < a.lower ? a.lower : sj;
  }
  __syncthreads();
  if (j == 0) {
    st->i += 1;
    st->p1 *= a.beta1;
    st->p2 *= a.beta2;
  }
}

// Sampled (COO) variant of the objective decision, on an estimate *F that
// holds mu/2 ||s||^2 already.  One workgroup of 64 threads.
template <typename T>
__global__ void ts_decide_from(TsArgs<T> a, const T* F, int init) {
  __shared__ T sh_s[kMaxRank];
  __shared__ int sh_roll;
  if (a.st->done) return;
  if ((int)threadIdx.x < a.R) sh_s[threadIdx.x] = a.s[threadIdx.x];
  if (threadIdx.x == 0) sh_roll = ts_decide(a, *F, init != 0);
  __syncthreads();
  if (!init) ts_keep_or_undo(a, sh_roll, sh_s);
}

// Copies A^(1..3) (rows of R values) into rows of RK values, zeros past R.
template <typename T>
__global__ void ts_pad(const T* __restrict__ A1, const T* __restrict__ A2, const T* __restrict__ A3, T* __restrict__ P,
                       int I1, int I2, int I3, int R, int RK) {
  const int64_t n = ((int64_t)I1 + I2 + I3) * RK;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / RK;
    const int j = (int)(e - row * RK);
    const T* A = row < I1 ? A1 : (row < I1 + I2 ? A2 : A3);
    const int64_t i = row < I1 ? row : (row < I1 + I2 ? row - I1 : row - I1 - I2);
    P[e] = j < R ? A[i * R + j] : T(0);
  }
}

template <typename T>
__global__ void ts_init(T* s, T* u, T* v, T* so, T* uo, T* vo, int R, TsgdState* st, double alpha) {
  const int j = threadIdx.x;
  if (j < R) s[j] = u[j] = v[j] = so[j] = uo[j] = vo[j] = T(0);
  if (j == 0) {
    st->F = 0.0;
    st->alpha = alpha;
    st->i = 0;
    st->p1 = 1.0;
    st->p2 = 1.0;
    st->rolled = 0ull;
    st->done = 0;
    st->epoch = 0;
  }
}

struct TsGeom {
  int nchunk, rows_per_grp, nblk;
};

TsGeom ts_geom(int I1, int I2, int I3) {
  TsGeom g;
  g.nchunk = (I3 + 63) / 64;
  const int64_t nrows = (int64_t)I1 * I2;
  const int64_t want_grp = std::max<int64_t>(1, kTsTargetBlocks / g.nchunk);
  g.rows_per_grp = (int)std::max<int64_t>(1, (nrows + want_grp - 1) / want_grp);
  const int64_t ngrp = (nrows + g.rows_per_grp - 1) / g.rows_per_grp;
  g.nblk = (int)(ngrp * g.nchunk);
  return g;
}

// Threads per workgroup: 512 while the per-lane arrays fit 256 registers.
template <typename T, int RK>
constexpr int ts_threads() { return sizeof(T) * RK <= 128 ? 512 : 256; }

template <typename T, int LOSS, int RK>
void ts_launch_mode(int mode, const TsArgs<T>& a, hipStream_t st) {
  constexpr int NT = ts_threads<T, RK>();
  if (mode == kTsGrad) {
    hipLaunchKernelGGL((ts_pass<T, LOSS, RK, kTsGrad, NT>), dim3(a.nblk), dim3(NT), 0, st, a);
    hipLaunchKernelGGL((ts_final<T, RK, kTsGrad, 512>), dim3(1), dim3(512), 0, st, a);
  } else if (mode == kTsObjInit) {
    hipLaunchKernelGGL((ts_pass<T, LOSS, RK, kTsObjInit, NT>), dim3(a.nblk), dim3(NT), 0, st, a);
    hipLaunchKernelGGL((ts_final<T, RK, kTsObjInit, 512>), dim3(1), dim3(512), 0, st, a);
  } else {
    hipLaunchKernelGGL((ts_pass<T, LOSS, RK, kTsObjEpoch, NT>), dim3(a.nblk), dim3(NT), 0, st, a);
    hipLaunchKernelGGL((ts_final<T, RK, kTsObjEpoch, 512>), dim3(1), dim3(512), 0, st, a);
  }
}

// Rank tile of the kernels for rank R.
int ts_rank_tile(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64; }

template <typename T, int LOSS>
void ts_launch_loss(int mode, const TsArgs<T>& a, hipStream_t st) {
  if (a.R <= 8)
    ts_launch_mode<T, LOSS, 8>(mode, a, st);
  else if (a.R <= 16)
    ts_launch_mode<T, LOSS, 16>(mode, a, st);
  else if (a.R <= 32)
    ts_launch_mode<T, LOSS, 32>(mode, a, st);
  else
    ts_launch_mode<T, LOSS, 64>(mode, a, st);
}

template <typename T>
void ts_launch(int loss, int mode, const TsArgs<T>& a, hipStream_t st) {
  if (loss == kGaussian)
    ts_launch_loss<T, kGaussian>(mode, a, st);
  else if (loss == kPoissonLog)
    ts_launch_loss<T, kPoissonLog>(mode, a, st);
  else if (loss == kBernoulliLogit)
    ts_launch_loss<T, kBernoulliLogit>(mode, a, st);
  else if (loss == kPoissonId)
    ts_launch_loss<T, kPoissonId>(mode, a, st);
  else
    ts_launch_loss<T, kBernoulliOdds>(mode, a, st);
}

size_t ts_vec_bytes(int R, size_t es) { return align_up((size_t)R * es, 64); }

// Workspace: state (256 B), u, v, s_o, u_o, v_o, padded factors, partial slots.
size_t ts_pad_off(int R, size_t es) { return align_up(256 + 5 * ts_vec_bytes(R, es), 256); }
size_t ts_part_off(int I1, int I2, int I3, int R, size_t es) {
  return ts_pad_off(R, es) + align_up(((size_t)I1 + I2 + I3) * ts_rank_tile(R) * es, 256);
}

template <typename T>
TsArgs<T> ts_args(const TsgdCall& c) {
  const TsGeom g = ts_geom(c.I1, c.I2, c.I3);
  char* base = static_cast<char*>(c.ws);
  const size_t vb = ts_vec_bytes(c.R, sizeof(T));
  TsArgs<T> a;
  a.X = static_cast<const T*>(c.X);
  const int RK = ts_rank_tile(c.R);
  T* pad = reinterpret_cast<T*>(base + ts_pad_off(c.R, sizeof(T)));
  a.A1 = pad;
  a.A2 = pad + (size_t)c.I1 * RK;
  a.A3 = pad + ((size_t)c.I1 + c.I2) * RK;
  a.s = static_cast<T*>(c.s);
  a.st = reinterpret_cast<TsgdState*>(base);
  char* vec = base + 256;
  a.u = reinterpret_cast<T*>(vec);
  a.v = reinterpret_cast<T*>(vec + vb);
  a.so = reinterpret_cast<T*>(vec + 2 * vb);
  a.uo = reinterpret_cast<T*>(vec + 3 * vb);
  a.vo = reinterpret_cast<T*>(vec + 4 * vb);
  a.part = reinterpret_cast<T*>(base + ts_part_off(c.I1, c.I2, c.I3, c.R, sizeof(T)));
  a.status = c.status;
  a.I1 = c.I1;
  a.I2 = c.I2;
  a.I3 = c.I3;
  a.R = c.R;
  a.nchunk = g.nchunk;
  a.rows_per_grp = g.rows_per_grp;
  a.nblk = g.nblk;
  a.tau = c.tau;
  a.mu = (T)c.mu;
  a.lower = c.lower == -INFINITY ? T(-INFINITY) : (T)c.lower;
  a.b1 = (T)c.beta1;
  a.b2 = (T)c.beta2;
  a.eps = (T)c.eps;
  a.beta1 = c.beta1;
  a.beta2 = c.beta2;
  a.tol = c.tol;
  return a;
}

template <typename T>
hipError_t ts_run(const TsgdCall& c) {
  TsArgs<T> a = ts_args<T>(c);
  char* base = static_cast<char*>(c.ws);
  const int RK = ts_rank_tile(c.R);
  T* pad = reinterpret_cast<T*>(base + ts_pad_off(c.R, sizeof(T)));
  const int64_t npad = ((int64_t)c.I1 + c.I2 + c.I3) * RK;
  hipLaunchKernelGGL(ts_pad<T>, dim3((unsigned)std::min<int64_t>(1024, (npad + 255) / 256)), dim3(256), 0, c.stream,
                     static_cast<const T*>(c.A[0]), static_cast<const T*>(c.A[1]), static_cast<const T*>(c.A[2]),
                     pad, c.I1, c.I2, c.I3, c.R, RK);
  hipLaunchKernelGGL(ts_init<T>, dim3(1), dim3(64), 0, c.stream, a.s, a.u, a.v, a.so, a.uo, a.vo, c.R, a.st,
                     c.alpha);
  ts_launch<T>(c.loss, kTsObjInit, a, c.stream);
  for (int e = 0; e < c.kappa; ++e) {
    for (int it = 0; it < c.tau; ++it) ts_launch<T>(c.loss, kTsGrad, a, c.stream);
    ts_launch<T>(c.loss, kTsObjEpoch, a, c.stream);
  }
  return hipGetLastError();
}

}  // namespace

size_t tsgd_ws_bytes(int I1, int I2, int I3, int R, int dtype) {
  const size_t es = dtype ? 8 : 4;
  const TsGeom g = ts_geom(I1, I2, I3);
  return ts_part_off(I1, I2, I3, R, es) + align_up((size_t)g.nblk * (R + 1) * es, 256);
}

hipError_t tsgd_run(const TsgdCall& c) { return c.dtype ? ts_run<double>(c) : ts_run<float>(c); }

hipError_t tsgd_sampled_begin(const TsgdCall& c) {
  if (c.dtype) {
    TsArgs<double> a = ts_args<double>(c);
    hipLaunchKernelGGL(ts_init<double>, dim3(1), dim3(64), 0, c.stream, a.s, a.u, a.v, a.so, a.uo, a.vo, c.R, a.st,
                       c.alpha);
  } else {
    TsArgs<float> a = ts_args<float>(c);
    hipLaunchKernelGGL(ts_init<float>, dim3(1), dim3(64), 0, c.stream, a.s, a.u, a.v, a.so, a.uo, a.vo, c.R, a.st,
                       c.alpha);
  }
  return hipGetLastError();
}

hipError_t tsgd_sampled_step(const TsgdCall& c, const void* g) {
  if (c.dtype)
    hipLaunchKernelGGL(ts_step_from<double>, dim3(1), dim3(64), 0, c.stream, ts_args<double>(c),
                       static_cast<const double*>(g));
  else
    hipLaunchKernelGGL(ts_step_from<float>, dim3(1), dim3(64), 0, c.stream, ts_args<float>(c),
                       static_cast<const float*>(g));
  return hipGetLastError();
}

hipError_t tsgd_sampled_decide(const TsgdCall& c, const void* F, int init) {
  if (c.dtype)
    hipLaunchKernelGGL(ts_decide_from<double>, dim3(1), dim3(64), 0, c.stream, ts_args<double>(c),
                       static_cast<const double*>(F), init);
  else
    hipLaunchKernelGGL(ts_decide_from<float>, dim3(1), dim3(64), 0, c.stream, ts_args<float>(c),
                       static_cast<const float*>(F), init);
  return hipGetLastError();
}

}  // namespace gcp
