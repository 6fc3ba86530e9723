// Unfused baseline of the same objective and gradient (FP32 only).
//
// The straightforward GPU formulation of Section 2.2 applied slice by slice:
// for each slice h of {t} u H_t
//   K_model  writes the full model tensor M_h  (eq. CP_model)
//   K_elem   reads X_h and M_h, writes Y_h = c_h df/dm and loss partials
//   K_mode1  G^(1) += Y_h(1) Z_1 diag(s_h)   (partial rows: a workgroup per
//            row i1 and chunk of its (i2,i3) entries)
//   K_mode2  G^(2) += Y_h(2) Z_2 diag(s_h)   (likewise per row i2)
//   K_mode3  partial rows of Y_h(3) Z_3 diag(s_h) per chunk of (i1,i2) pairs
//   K_gs     (current slice) partials of Z^T vec(Y_t)
// then one kernel sums the partials and adds the regularisation terms.
// Every accumulation has a single owner, so results are deterministic.
#include "common.hpp"

namespace gcp {
namespace {

constexpr int kPairChunk = 64;

struct PlainLayout {
  size_t M, Y, g1p, g2p, g3p, gsp, lossp, total;
  int nchunks, eblocks, split1, split2;
};

constexpr int kEBlocks = 1024;

// Chunks per row of the mode-1 and mode-2 products: enough workgroups to
// fill the device (about 2048), each chunk at least 1024 entries.
int row_split(int rows, size_t per_row) {
  const size_t want = (2048 + (size_t)rows - 1) / (size_t)rows;
  const size_t cap = std::max<size_t>(1, per_row / 1024);
  return (int)std::max<size_t>(1, std::min(want, cap));
}

PlainLayout plain_layout(int I1, int I2, int I3, int R) {
  PlainLayout p;
  size_t omega = (size_t)I1 * I2 * I3;
  p.nchunks = (int)(((size_t)I1 * I2 + kPairChunk - 1) / kPairChunk);
  p.eblocks = kEBlocks;
  p.split1 = row_split(I1, (size_t)I2 * I3);
  p.split2 = row_split(I2, (size_t)I1 * I3);
  size_t off = 0;
  p.M = off; off = align_up(off + omega * 4, 256);
  p.Y = off; off = align_up(off + omega * 4, 256);
  p.g1p = off; off = align_up(off + (size_t)p.split1 * I1 * R * 4, 256);
  p.g2p = off; off = align_up(off + (size_t)p.split2 * I2 * R * 4, 256);
  p.g3p = off; off = align_up(off + (size_t)p.nchunks * I3 * R * 4, 256);
  p.gsp = off; off = align_up(off + (size_t)p.nchunks * ((I3 + 255) / 256) * R * 4, 256);
  p.lossp = off; off = align_up(off + (size_t)kMaxNs * kEBlocks * 4, 256);
  p.total = off;
  return p;
}

__global__ void __launch_bounds__(256) k_model(const float* __restrict__ A1, const float* __restrict__ A2,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ M, int I2, int I3, int R, size_t omega) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < omega;
       e += (size_t)gridDim.x * blockDim.x) {
    size_t p = e / I3;
    int i3 = (int)(e - p * I3);
    int i1 = (int)(p / I2), i2 = (int)(p - (size_t)i1 * I2);
    float m = 0.f;
    for (int j = 0; j < R; ++j) m += s[j] * A1[(size_t)i1 * R + j] * A2[(size_t)i2 * R + j] * A3[(size_t)i3 * R + j];
    M[e] = m;
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

// Block reduction of RT per-thread values: wave sums, then the four waves in
// order; sm[j] holds the block sum of element j afterwards.
template <int RT>
__device__ void block_reduce_rows(float (&acc)[RT], float* sm /* 4*RT */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < RT; ++j) {
    float v = acc[j];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) sm[wave * RT + j] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < RT)
    sm[threadIdx.x] = ((sm[threadIdx.x] + sm[RT + threadIdx.x]) + sm[2 * RT + threadIdx.x]) + sm[3 * RT + threadIdx.x];
  __syncthreads();
}

// Partial row (i1, chunk blockIdx.y of its entries) of
// G^(1) (+)= sum_{i2,i3} Y[i1,i2,i3] A2[i2,:] A3[i3,:] s_h
template <int RT>
__global__ void __launch_bounds__(256) k_mode1(const float* __restrict__ Y, const float* __restrict__ A2,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ G1p, int I1, int I2, int I3, int R,
                                               int accumulate) {
  extern __shared__ float sm[];
  const int i1 = blockIdx.x;
  float acc[RT];
  for (int j = 0; j < RT; ++j) acc[j] = 0.f;
  const size_t n = (size_t)I2 * I3;
  const size_t e0 = n * blockIdx.y / gridDim.y, e1 = n * (blockIdx.y + 1) / gridDim.y;
  const float* row = Y + (size_t)i1 * n;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    int i2 = (int)(e / I3), i3 = (int)(e - (size_t)i2 * I3);
    float y = row[e];
    for (int j = 0; j < RT; ++j)
      if (j < R) acc[j] += y * A2[(size_t)i2 * R + j] * A3[(size_t)i3 * R + j];
  }
  block_reduce_rows<RT>(acc, sm);
  if ((int)threadIdx.x < R) {
    float v = sm[threadIdx.x] * s[threadIdx.x];
    float* g = G1p + ((size_t)blockIdx.y * I1 + i1) * R + threadIdx.x;
    *g = accumulate ? *g + v : v;
  }
}

// Partial row (i2, chunk blockIdx.y) of
// G^(2) (+)= sum_{i1,i3} Y[i1,i2,i3] A1[i1,:] A3[i3,:] s_h
template <int RT>
__global__ void __launch_bounds__(256) k_mode2(const float* __restrict__ Y, const float* __restrict__ A1,
                                               const float* __restrict__ A3, const float* __restrict__ s,
                                               float* __restrict__ G2p, int I1, int I2, int I3, int R,
                                               int accumulate) {
  extern __shared__ float sm[];
  const int i2 = blockIdx.x;
  float acc[RT];
  for (int j = 0; j < RT; ++j) acc[j] = 0.f;
  const size_t n = (size_t)I1 * I3;
  const size_t e0 = n * blockIdx.y / gridDim.y, e1 = n * (blockIdx.y + 1) / gridDim.y;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    int i1 = (int)(e / I3), i3 = (int)(e - (size_t)i1 * I3);
    float y = Y[((size_t)i1 * I2 + i2) * I3 + i3];
    for (int j = 0; j < RT; ++j)
      if (j < R) acc[j] += y * A1[(size_t)i1 * R + j] * A3[(size_t)i3 * R + j];
  }
  block_reduce_rows<RT>(acc, sm);
  if ((int)threadIdx.x < R) {
    float v = sm[threadIdx.x] * s[threadIdx.x];
    float* g = G2p + ((size_t)blockIdx.y * I2 + i2) * R + threadIdx.x;
    *g = accumulate ? *g + v : v;
  }
}

// Per chunk of kPairChunk pairs: partial G^(3) rows (thread per i3), and for
// the current slice the partial Z^T vec(Y_t).
template <int RT>
__global__ void __launch_bounds__(256) k_mode3(const float* __restrict__ Y, const float* __restrict__ A1,
                                               const float* __restrict__ A2, const float* __restrict__ A3,
                                               const float* __restrict__ s, float* __restrict__ g3p,
                                               float* __restrict__ gsp, int I1, int I2, int I3, int R,
                                               int accumulate) {
  extern __shared__ float sm[];
  const int chunk = blockIdx.x;
  const int i3 = blockIdx.y * 256 + threadIdx.x;
  const size_t p0 = (size_t)chunk * kPairChunk;
  const size_t npairs = (size_t)I1 * I2;
  float acc[RT], accs[RT];
  for (int j = 0; j < RT; ++j) acc[j] = accs[j] = 0.f;
  if (i3 < I3) {
    for (size_t p = p0; p < p0 + kPairChunk && p < npairs; ++p) {
      int i1 = (int)(p / I2), i2 = (int)(p - (size_t)i1 * I2);
      float y = Y[p * I3 + i3];
      for (int j = 0; j < RT; ++j) {
        if (j < R) {
          float w = A1[(size_t)i1 * R + j] * A2[(size_t)i2 * R + j];
          acc[j] += y * w;
          accs[j] += y * w * A3[(size_t)i3 * R + j];
        }
      }
    }
    for (int j = 0; j < R; ++j) {
      float* g = g3p + ((size_t)chunk * I3 + i3) * R + j;
      float v = acc[j] * s[j];
      *g = accumulate ? *g + v : v;
    }
  }
  if (gsp) {  // current slice only
    block_reduce_rows<RT>(accs, sm);
    if ((int)threadIdx.x < R) {
      float* g = gsp + ((size_t)chunk * gridDim.y + blockIdx.y) * R + threadIdx.x;
      *g = sm[threadIdx.x];
    }
  }
}

__global__ void __launch_bounds__(256) k_final(float* G1, float* G2, float* G3, float* gs, float* loss,
                                               const float* A1, const float* A2, const float* A3,
                                               const float* st, const float* g1p, const float* g2p,
                                               const float* g3p, const float* gsp, const float* lossp,
                                               int nloss, int I1, int I2, int I3, int R, int split1,
                                               int split2, int nchunks, int nygs, float lam, float mu,
                                               int want, int* status) {
  if ((int)blockIdx.x < (int)gridDim.x - 1) {
    const int n1 = I1 * R, n2 = I2 * R, n3 = I3 * R;
    const int total = n1 + n2 + n3 + R;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (gridDim.x - 1) * 256) {
      float out;
      if (idx < n1) {
        Kahan<float> k;
        for (int c = 0; c < split1; ++c) k.add(g1p[(size_t)c * n1 + idx]);
        out = k.s + lam * A1[idx];
        G1[idx] = out;
      } else if (idx < n1 + n2) {
        int e = idx - n1;
        Kahan<float> k;
        for (int c = 0; c < split2; ++c) k.add(g2p[(size_t)c * n2 + e]);
        out = k.s + lam * A2[e];
        G2[e] = out;
      } else if (idx < n1 + n2 + n3) {
        int e = idx - n1 - n2;
        Kahan<float> k;
        for (int c = 0; c < nchunks; ++c) k.add(g3p[(size_t)c * n3 + e]);
        out = k.s + lam * A3[e];
        G3[e] = out;
      } else {
        int j = idx - n1 - n2 - n3;
        Kahan<float> k;
        for (int c = 0; c < nchunks * nygs; ++c) k.add(gsp[(size_t)c * R + j]);
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
  const size_t shm = 4 * RT * sizeof(float);
  const int ygs = (c.I3 + 255) / 256;
  for (int h = 0; h < c.ns; ++h) {
    const float* X = static_cast<const float*>(c.X[h]);
    const size_t pitch = (h == 0 || c.ring_pitch == 0) ? (size_t)c.I3 : c.ring_pitch;
    const float* s = static_cast<const float*>(c.S[h]);
    hipLaunchKernelGGL(k_model, dim3(2048), dim3(256), 0, c.stream, A1, A2, A3, s, M, c.I2, c.I3, c.R, omega);
    float ch = (float)c.c[h];
    hipError_t e;
    switch (c.loss) {
      case kGaussian:
        hipLaunchKernelGGL(k_elem<kGaussian>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch, omega, c.I3,
                           pitch, lossp + (size_t)h * kEBlocks);
        break;
      case kPoissonLog:
        hipLaunchKernelGGL(k_elem<kPoissonLog>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch, omega, c.I3,
                           pitch, lossp + (size_t)h * kEBlocks);
        break;
      case kBernoulliLogit:
        hipLaunchKernelGGL(k_elem<kBernoulliLogit>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch,
                           omega, c.I3, pitch, lossp + (size_t)h * kEBlocks);
        break;
      case kPoissonId:
        hipLaunchKernelGGL(k_elem<kPoissonId>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch, omega, c.I3,
                           pitch, lossp + (size_t)h * kEBlocks);
        break;
      default:
        hipLaunchKernelGGL(k_elem<kBernoulliOdds>, dim3(kEBlocks), dim3(256), 0, c.stream, X, M, Y, ch,
                           omega, c.I3, pitch, lossp + (size_t)h * kEBlocks);
    }
    if (c.want & kWantGrad) {
      hipLaunchKernelGGL(k_mode1<RT>, dim3(c.I1, L.split1), dim3(256), shm, c.stream, Y, A2, A3, s, g1p, c.I1,
                         c.I2, c.I3, c.R, h > 0);
      hipLaunchKernelGGL(k_mode2<RT>, dim3(c.I2, L.split2), dim3(256), shm, c.stream, Y, A1, A3, s, g2p, c.I1,
                         c.I2, c.I3, c.R, h > 0);
      hipLaunchKernelGGL(k_mode3<RT>, dim3(L.nchunks, ygs), dim3(256), shm, c.stream, Y, A1, A2, A3, s, g3p,
                         h == 0 ? gsp : nullptr, c.I1, c.I2, c.I3, c.R, h > 0);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int total = (c.I1 + c.I2 + c.I3 + 1) * c.R;
  const int gblocks = (c.want & kWantGrad) ? std::min(1024, (total + 255) / 256) : 0;
  hipLaunchKernelGGL(k_final, dim3(gblocks + 1), dim3(256), 0, c.stream, G1, G2, G3, static_cast<float*>(c.gs),
                     static_cast<float*>(c.loss_out), A1, A2, A3, static_cast<const float*>(c.S[0]), g1p, g2p,
                     g3p, gsp, lossp, c.ns * kEBlocks, c.I1, c.I2, c.I3, c.R, L.split1, L.split2, L.nchunks,
                     ygs, (float)c.lam, (float)c.mu, c.want, c.status);
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
