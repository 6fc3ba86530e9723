// Unfused baseline of the same objective and gradient (FP32 only).
//
// The straightforward GPU formulation of Section 2.2 applied slice by slice,
// each step its own kernel with its result in device memory:
// for each slice h of {t} u H_t
//   K_model  writes the full model tensor M_h  (eq. CP_model)
//   K_elem   reads X_h and M_h, writes Y_h = c_h df/dm and loss partials
//   K_mode1  partial rows of G^(1) += Y_h(1) Z_1 diag(s_h)
//   K_mode2  partial rows of G^(2) += Y_h(2) Z_2 diag(s_h)
//   K_mode3  partial rows of G^(3) += Y_h(3) Z_3 diag(s_h), and for the current
//            slice the partial sums of Z^T vec(Y_t)
// then one kernel sums the partials in a fixed order and adds the
// regularisation terms.  About 28 bytes of HBM traffic per entry and slice
// (X read, M written and read, Y written and read three times) against the
// fused kernel's 4.
//
// Each product kernel is written to stream at the memory rate: a 64-thread
// block owns 64 consecutive i3 (a lane keeps its A3 row in registers), walks
// a run of (i1, i2) rows reading 256 contiguous bytes per row, and takes the
// per-row factor values (W = s A1 A2, or A1 / A2 alone) from LDS or as
// wave-uniform loads.  Every partial has a single owner, so the results are
// deterministic.
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kPB = 64;        // threads per block (one wave): consecutive i3
constexpr int kRows = 64;      // (i1, i2) rows per model / mode-3 block
constexpr int kEBlocks = 1024;

struct PlainLayout {
  size_t M, Y, g1p, g2p, g3p, gsp, lossp, total;
  int nc3;        // i3 chunks of kPB
  int nrow3;      // row runs of the model / mode-3 kernels (kRows rows each)
  int s1, s2;     // chunks of the inner mode of the mode-1 / mode-2 products
};

// chunks of the inner mode of the mode-1 / mode-2 products: enough blocks
// (about 2048 with the i3 chunks), at least 8 rows each
int inner_split(int rows, int other, int nc3) {
  const int want = std::max(1, 2048 / std::max(1, rows * nc3));
  return std::max(1, std::min(want, other / 8));
}

PlainLayout plain_layout(int I1, int I2, int I3, int R) {
  PlainLayout p;
  size_t omega = (size_t)I1 * I2 * I3;
  p.nc3 = (I3 + kPB - 1) / kPB;
  p.nrow3 = (int)(((size_t)I1 * I2 + kRows - 1) / kRows);
  p.s1 = inner_split(I1, I2, p.nc3);
  p.s2 = inner_split(I2, I1, p.nc3);
  size_t off = 0;
  p.M = off; off = align_up(off + omega * 4, 256);
  p.Y = off; off = align_up(off + omega * 4, 256);
  p.g1p = off; off = align_up(off + (size_t)p.s1 * p.nc3 * I1 * R * 4, 256);
  p.g2p = off; off = align_up(off + (size_t)p.s2 * p.nc3 * I2 * R * 4, 256);
  p.g3p = off; off = align_up(off + (size_t)p.nrow3 * I3 * R * 4, 256);
  p.gsp = off; off = align_up(off + (size_t)p.nrow3 * p.nc3 * R * 4, 256);
  p.lossp = off; off = align_up(off + (size_t)kMaxNs * kEBlocks * 4, 256);
  p.total = off;
  return p;
}

// A3 row of this lane's i3 (zero past I3 and past R)
template <int RT>
__device__ __forceinline__ void a3_row(const float* __restrict__ A3, int i3, int I3, int R, float (&a3)[RT]) {
#pragma unroll
  for (int j = 0; j < RT; ++j) a3[j] = (i3 < I3 && j < R) ? A3[(size_t)i3 * R + j] : 0.f;
}

// Sum over the block's 64 lanes of RT per-lane values; lane j ends with
// element j (RT <= 64).
template <int RT>
__device__ __forceinline__ float block_sum(float (&v)[RT], float* sm /* RT x 65 */) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int j = 0; j < RT; ++j) sm[j * 65 + lane] = v[j];
  __syncthreads();
  float s = 0.f;
  if (lane < RT)
    for (int l = 0; l < kPB; ++l) s += sm[lane * 65 + l];
  __syncthreads();
  return s;
}

// W = s A1[i1] A2[i2] (or A1 A2 without s) of kRows rows, into LDS
template <int RT>
__device__ __forceinline__ void row_weights(float (*W)[RT], const float* __restrict__ A1,
                                            const float* __restrict__ A2, const float* __restrict__ s,
                                            size_t row0, size_t nrows, int I2, int R) {
  for (int idx = threadIdx.x; idx < kRows * RT; idx += kPB) {
    const int q = idx / RT, j = idx % RT;
    const size_t row = row0 + q;
    float w = 0.f;
    if (row < nrows && j < R) {
      const int i1 = (int)(row / I2), i2 = (int)(row - (size_t)i1 * I2);
      w = A1[(size_t)i1 * R + j] * A2[(size_t)i2 * R + j];
      if (s) w *= s[j];
    }
    W[q][j] = w;
  }
  __syncthreads();
}

// M[row, i3] = sum_j W[row, j] A3[i3, j], W = s A1[i1] A2[i2], for kRows rows
template <int RT>
__global__ void __launch_bounds__(kPB) k_model(const float* __restrict__ A1, const float* __restrict__ A2,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ M, int I1, int I2, int I3, int R) {
  __shared__ float W[kRows][RT];
  const int i3 = blockIdx.x * kPB + threadIdx.x;
  const size_t row0 = (size_t)blockIdx.y * kRows;
  const size_t nrows = (size_t)I1 * I2;
  row_weights<RT>(W, A1, A2, s, row0, nrows, I2, R);
  float a3[RT];
  a3_row<RT>(A3, i3, I3, R, a3);
  if (i3 >= I3) return;
  for (int q = 0; q < kRows && row0 + q < nrows; ++q) {
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < RT; ++j) m = fmaf(W[q][j], a3[j], m);
    M[(row0 + q) * I3 + i3] = m;
  }
}

template <int LOSS>
__global__ void __launch_bounds__(256) k_elem(const float* __restrict__ X, const float* __restrict__ M,
                                              float* __restrict__ Y, float ch, size_t omega, int I3,
                                              size_t pitch, float* __restrict__ lossp) {
  __shared__ float red[256];
  Kahan<float> k;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < omega;
       e += (size_t)gridDim.x * blockDim.x) {
    // X rows may be padded (stored slices): element e is row e / I3
    size_t xe = e;
    if (pitch != (size_t)I3) {
      const size_t pr = e / (size_t)I3;
      xe = pr * pitch + (e - pr * (size_t)I3);
    }
    float f, y;
    LossFn<float, LOSS>::eval(X[xe], M[e], f, y);
    Y[e] = ch * y;
    k.add(ch * f);
  }
  red[threadIdx.x] = k.s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0];
}

// Partial row i1 (blockIdx.z) of G^(1) over the i2 chunk blockIdx.y and the
// i3 chunk blockIdx.x: sum_{i2,i3} Y[i1,i2,i3] A2[i2,:] A3[i3,:] s_h, in slot
// (chunk y, chunk x); `accumulate` adds to the slot (later slices).
template <int RT>
__global__ void __launch_bounds__(kPB) k_mode1(const float* __restrict__ Y, const float* __restrict__ A2,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ G1p, int I1, int I2, int I3, int R, int nc3,
                                               int accumulate) {
  __shared__ float sm[RT * 65];
  const int i1 = blockIdx.z, i3 = blockIdx.x * kPB + threadIdx.x;
  const int a0 = (int)((size_t)I2 * blockIdx.y / gridDim.y), a1 = (int)((size_t)I2 * (blockIdx.y + 1) / gridDim.y);
  float t[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) t[j] = 0.f;
  if (i3 < I3) {
    const float* yrow = Y + (size_t)i1 * I2 * I3 + i3;
    for (int i2 = a0; i2 < a1; ++i2) {
      const float y = yrow[(size_t)i2 * I3];
      const float* a2 = A2 + (size_t)i2 * R;
#pragma unroll
      for (int j = 0; j < RT; ++j) t[j] = fmaf(y, j < R ? a2[j] : 0.f, t[j]);
    }
  }
  float a3[RT];
  a3_row<RT>(A3, i3, I3, R, a3);
#pragma unroll
  for (int j = 0; j < RT; ++j) t[j] *= a3[j];
  const float v = block_sum<RT>(t, sm);
  if ((int)threadIdx.x < R) {
    float* g = G1p + (((size_t)blockIdx.y * nc3 + blockIdx.x) * I1 + i1) * R + threadIdx.x;
    const float out = v * s[threadIdx.x];
    *g = accumulate ? *g + out : out;
  }
}

// Partial row i2 (blockIdx.z) of G^(2) over the i1 chunk blockIdx.y and the
// i3 chunk blockIdx.x.
template <int RT>
__global__ void __launch_bounds__(kPB) k_mode2(const float* __restrict__ Y, const float* __restrict__ A1,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ G2p, int I1, int I2, int I3, int R, int nc3,
                                               int accumulate) {
  __shared__ float sm[RT * 65];
  const int i2 = blockIdx.z, i3 = blockIdx.x * kPB + threadIdx.x;
  const int a0 = (int)((size_t)I1 * blockIdx.y / gridDim.y), a1 = (int)((size_t)I1 * (blockIdx.y + 1) / gridDim.y);
  float t[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) t[j] = 0.f;
  if (i3 < I3) {
    for (int i1 = a0; i1 < a1; ++i1) {
      const float y = Y[((size_t)i1 * I2 + i2) * I3 + i3];
      const float* r1 = A1 + (size_t)i1 * R;
#pragma unroll
      for (int j = 0; j < RT; ++j) t[j] = fmaf(y, j < R ? r1[j] : 0.f, t[j]);
    }
  }
  float a3[RT];
  a3_row<RT>(A3, i3, I3, R, a3);
#pragma unroll
  for (int j = 0; j < RT; ++j) t[j] *= a3[j];
  const float v = block_sum<RT>(t, sm);
  if ((int)threadIdx.x < R) {
    float* g = G2p + (((size_t)blockIdx.y * nc3 + blockIdx.x) * I2 + i2) * R + threadIdx.x;
    const float out = v * s[threadIdx.x];
    *g = accumulate ? *g + out : out;
  }
}

// Per run of kRows (i1, i2) rows: partial G^(3) rows (lane per i3), and for
// the current slice the partial Z^T vec(Y_t) = sum_i3 A3[i3,:] (partial row).
template <int RT>
__global__ void __launch_bounds__(kPB) k_mode3(const float* __restrict__ Y, const float* __restrict__ A1,
                                               const float* __restrict__ A2, const float* __restrict__ A3,
                                               const float* __restrict__ s, float* __restrict__ g3p,
                                               float* __restrict__ gsp, int I1, int I2, int I3, int R,
                                               int accumulate) {
  __shared__ float W[kRows][RT];
  __shared__ float sm[RT * 65];
  const int i3 = blockIdx.x * kPB + threadIdx.x;
  const size_t row0 = (size_t)blockIdx.y * kRows;
  const size_t nrows = (size_t)I1 * I2;
  row_weights<RT>(W, A1, A2, nullptr, row0, nrows, I2, R);
  float acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc[j] = 0.f;
  if (i3 < I3) {
    for (int q = 0; q < kRows && row0 + q < nrows; ++q) {
      const float y = Y[(row0 + q) * I3 + i3];
#pragma unroll
      for (int j = 0; j < RT; ++j) acc[j] = fmaf(y, W[q][j], acc[j]);
    }
    for (int j = 0; j < R; ++j) {
      float* g = g3p + ((size_t)blockIdx.y * I3 + i3) * R + j;
      const float v = acc[j] * s[j];
      *g = accumulate ? *g + v : v;
    }
  }
  if (gsp) {  // current slice only
    float a3[RT];
    a3_row<RT>(A3, i3, I3, R, a3);
#pragma unroll
    for (int j = 0; j < RT; ++j) acc[j] *= a3[j];
    const float v = block_sum<RT>(acc, sm);
    if ((int)threadIdx.x < R) gsp[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * R + threadIdx.x] = v;
  }
}

__global__ void __launch_bounds__(256) k_final(float* G1, float* G2, float* G3, float* gs, float* loss,
                                               const float* A1, const float* A2, const float* A3,
                                               const float* st, const float* g1p, const float* g2p,
                                               const float* g3p, const float* gsp, const float* lossp,
                                               int nloss, int I1, int I2, int I3, int R, int n1slots,
                                               int n2slots, int n3slots, int ngsslots, float lam, float mu,
                                               int want, int* status) {
  if ((int)blockIdx.x < (int)gridDim.x - 1) {
    const int n1 = I1 * R, n2 = I2 * R, n3 = I3 * R;
    const int total = n1 + n2 + n3 + R;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (gridDim.x - 1) * 256) {
      float out;
      Kahan<float> k;
      if (idx < n1) {
        for (int c = 0; c < n1slots; ++c) k.add(g1p[(size_t)c * n1 + idx]);
        out = k.s + lam * A1[idx];
        G1[idx] = out;
      } else if (idx < n1 + n2) {
        const int e = idx - n1;
        for (int c = 0; c < n2slots; ++c) k.add(g2p[(size_t)c * n2 + e]);
        out = k.s + lam * A2[e];
        G2[e] = out;
      } else if (idx < n1 + n2 + n3) {
        const int e = idx - n1 - n2;
        for (int c = 0; c < n3slots; ++c) k.add(g3p[(size_t)c * n3 + e]);
        out = k.s + lam * A3[e];
        G3[e] = out;
      } else {
        const int j = idx - n1 - n2 - n3;
        for (int c = 0; c < ngsslots; ++c) k.add(gsp[(size_t)c * R + j]);
        out = k.s + mu * st[j];
        gs[j] = out;
      }
      if (!isfinite(out)) atomicOr(status, (int)kStatusNonFinite);
    }
    return;
  }
  if (!(want & kWantLoss)) return;
  __shared__ float red[256];
  Kahan<float> k;
  for (int b = threadIdx.x; b < nloss; b += 256) k.add(lossp[b]);
  const float* mats[3] = {A1, A2, A3};
  const int rows[3] = {I1, I2, I3};
  Kahan<float> kr;
  for (int m = 0; m < 3; ++m)
    for (int e = threadIdx.x; e < rows[m] * R; e += 256) kr.add(mats[m][e] * mats[m][e]);
  Kahan<float> ks;
  for (int j = threadIdx.x; j < R; j += 256) ks.add(st[j] * st[j]);
  red[threadIdx.x] = k.s + 0.5f * lam * kr.s + 0.5f * mu * ks.s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    loss[0] = red[0];
    if (!isfinite(red[0])) atomicOr(status, (int)kStatusNonFinite);
  }
}

template <int LOSS>
void launch_elem(const DenseCall& c, const float* X, const float* M, float* Y, float ch, size_t omega, size_t pitch,
                 float* lp) {
  hipLaunchKernelGGL(k_elem<LOSS>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch, omega, c.I3, pitch, lp);
}

template <int RT>
hipError_t run_rt(const DenseCall& c, char* base, const PlainLayout& L) {
  const size_t omega = (size_t)c.I1 * c.I2 * c.I3;
  float* M = reinterpret_cast<float*>(base + L.M);
  float* Y = reinterpret_cast<float*>(base + L.Y);
  float* g1p = reinterpret_cast<float*>(base + L.g1p);
  float* g2p = reinterpret_cast<float*>(base + L.g2p);
  float* g3p = reinterpret_cast<float*>(base + L.g3p);
  float* gsp = reinterpret_cast<float*>(base + L.gsp);
  float* lossp = reinterpret_cast<float*>(base + L.lossp);
  const float* A1 = static_cast<const float*>(c.A[0]);
  const float* A2 = static_cast<const float*>(c.A[1]);
  const float* A3 = static_cast<const float*>(c.A[2]);
  float* G1 = static_cast<float*>(c.G[0]);
  float* G2 = static_cast<float*>(c.G[1]);
  float* G3 = static_cast<float*>(c.G[2]);
  const dim3 g_rows((unsigned)L.nc3, (unsigned)L.nrow3);
  for (int h = 0; h < c.ns; ++h) {
    const float* X = static_cast<const float*>(c.X[h]);
    const size_t pitch = (h == 0 || c.ring_pitch == 0) ? (size_t)c.I3 : c.ring_pitch;
    const float* s = static_cast<const float*>(c.S[h]);
    hipLaunchKernelGGL(k_model<RT>, g_rows, dim3(kPB), 0, c.stream, A1, A2, A3, s, M, c.I1, c.I2, c.I3, c.R);
    const float ch = (float)c.c[h];
    float* lp = lossp + (size_t)h * kEBlocks;
    switch (c.loss) {
      case kGaussian: launch_elem<kGaussian>(c, X, M, Y, ch, omega, pitch, lp); break;
      case kPoissonLog: launch_elem<kPoissonLog>(c, X, M, Y, ch, omega, pitch, lp); break;
      case kBernoulliLogit: launch_elem<kBernoulliLogit>(c, X, M, Y, ch, omega, pitch, lp); break;
      case kPoissonId: launch_elem<kPoissonId>(c, X, M, Y, ch, omega, pitch, lp); break;
      default: launch_elem<kBernoulliOdds>(c, X, M, Y, ch, omega, pitch, lp);
    }
    if (c.want & kWantGrad) {
      hipLaunchKernelGGL(k_mode1<RT>, dim3((unsigned)L.nc3, (unsigned)L.s1, (unsigned)c.I1), dim3(kPB), 0, c.stream, Y,
                         A2, A3, s, g1p, c.I1, c.I2, c.I3, c.R, L.nc3, h > 0);
      hipLaunchKernelGGL(k_mode2<RT>, dim3((unsigned)L.nc3, (unsigned)L.s2, (unsigned)c.I2), dim3(kPB), 0, c.stream, Y,
                         A1, A3, s, g2p, c.I1, c.I2, c.I3, c.R, L.nc3, h > 0);
      hipLaunchKernelGGL(k_mode3<RT>, g_rows, dim3(kPB), 0, c.stream, Y, A1, A2, A3, s, g3p, h == 0 ? gsp : nullptr,
                         c.I1, c.I2, c.I3, c.R, h > 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int total = (c.I1 + c.I2 + c.I3 + 1) * c.R;
  const int gblocks = (c.want & kWantGrad) ? std::min(1024, (total + 255) / 256) : 0;
  hipLaunchKernelGGL(k_final, dim3(gblocks + 1), dim3(256), 0, c.stream, G1, G2, G3, static_cast<float*>(c.gs),
                     static_cast<float*>(c.loss_out), A1, A2, A3, static_cast<const float*>(c.S[0]), g1p, g2p, g3p,
                     gsp, lossp, c.ns * kEBlocks, c.I1, c.I2, c.I3, c.R, L.s1 * L.nc3, L.s2 * L.nc3, L.nrow3,
                     L.nrow3 * L.nc3, (float)c.lam, (float)c.mu, c.want, c.status);
  return hipGetLastError();
}

}  // namespace

size_t dense_plain_scratch_bytes(int I1, int I2, int I3, int R, int dtype) {
  (void)dtype;
  return plain_layout(I1, I2, I3, R).total;
}

hipError_t dense_plain_run(const DenseCall& c, void* scratch, size_t scratch_bytes) {
  if (c.dtype != 0) return hipErrorInvalidValue;
  PlainLayout L = plain_layout(c.I1, c.I2, c.I3, c.R);
  if (L.total > scratch_bytes) return hipErrorInvalidValue;
  char* base = static_cast<char*>(scratch);
  if (c.R <= 4) return run_rt<4>(c, base, L);
  if (c.R <= 8) return run_rt<8>(c, base, L);
  if (c.R <= 16) return run_rt<16>(c, base, L);
  if (c.R <= 32) return run_rt<32>(c, base, L);
  return run_rt<64>(c, base, L);
}

}  // namespace gcp
