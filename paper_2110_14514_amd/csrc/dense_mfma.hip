// Fused objective/gradient over a dense slice and its window, with the two
// rank-R contractions on the FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Same quantities as the VALU kernel (eq. gcp_stream_problem_1 and the
// gradients of Section 4.2), organised around two small GEMMs per group of
// 64 entries e of one (i1,i2) pair row:
//   GEMM1  m[h][e]  = sum_j S[h][j] P[e][j],  P[e][j] = A1[i1,j] A2[i2,j] A3[i3,j]
//   GEMM2  yhat[j][e] = sum_h S[h][j] c_h y(x_he, m[h][e])
// (h runs over the current slice and the stored window, S[h] = s_h).  With
// the 16x16x4 lane layout the accumulator of GEMM1 (rows h, columns e) is
// directly the B operand of GEMM2 (K = h), so the loss derivative is applied
// in registers between the two and nothing is staged through memory.
// The mode products that follow are elementwise in j and stay on the VALU:
//   G3[i3,:]  += yhat[:,e] * A1[i1,:] * A2[i2,:]      (lane-local)
//   V[i1,i2,:] = sum_i3 yhat[:,e] * A3[i3,:]          (16-lane reduce-scatter)
//   G1[i1,:] += V * A2[i2,:],  G2[i2,:] += V * A1[i1,:]
//   g_s      += y_t[e] * P[e,:]                       (current slice only)
//
// Lane layout of the 16x16x4 FP32 MFMA (lane l = 16 g + n):
//   A operand: A[row n][k g];  B operand: B[k g][col n];
//   accumulator register r: D[row 4g + r][col n].
// GEMM1: rows = h (16 per h-tile), cols = 16 entries, K = j.  The K index of
// step t held by lane group g is j(t,g) = 16 (t/4) + 4g + t%4, chosen so that
// GEMM2's output row of register r in M-tile mt, j = 16 mt + 4g + r, is the
// same j a lane already holds for step t = 4 mt + r.
// Entries: a full group is NU 16-column tiles u (NU = 4 at rank 16, 2 at
// rank 32, to fit the register file) with i3 = c0 + NU n + u, so each lane
// loads NU contiguous values per slice; the ragged tail of a row uses
// i3 = c0 + 16u + n with only the tiles that hold entries.
//
// Work decomposition: each wave owns a TB1 x TB2 block of pairs over all of
// I3; eight waves form a workgroup that combines its waves' mode-3 rows and
// temporal-gradient partials in a fixed order.  All partials go to
// block/workgroup-indexed slots and are summed in a fixed order by the
// reduce kernel, so results are bitwise reproducible.
#include "common.hpp"

namespace gcp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kTB = 32;

struct MArgs {
  const float* X[kMaxNs];
  const float* S[kMaxNs];
  float c[kMaxNs];
  const float* A1;
  const float* A2;
  const float* A3;
  float* G1p;
  float* G2p;
  float* G3p;
  float* gsp;
  float* lossp;
  int I1, I2, I3, R, ns, want, tb1, tb2, nb2, nblocks;
};

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NT>
__device__ __forceinline__ float row_reduce_scatter(float (&v)[NT], int n) {
  // sum over the 16 lanes of a row; lane n ends with element n >> (4 - log2 NT)
  int mask = 8;
#pragma unroll
  for (int half = NT / 2; half >= 1; half /= 2) {
    const bool hi = (n & mask) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      float send = hi ? v[i] : v[i + half];
      float keep = hi ? v[i + half] : v[i];
      v[i] = keep + __shfl_xor(send, mask);
    }
    mask >>= 1;
  }
  float r = v[0];
  for (; mask >= 1; mask >>= 1) r += __shfl_xor(r, mask);
  return r;
}

template <int LOSS, int RT, int NH>
__global__ void __launch_bounds__(kThreads) fused_dense_mfma(MArgs a) {
  constexpr int NT = RT / 4;   // K steps of GEMM1 = j slots per lane
  constexpr int NM = RT / 16;  // M tiles of GEMM2
  constexpr int LOGNT = NT == 4 ? 2 : 3;
  constexpr int NU = RT == 32 ? 2 : 4;  // 16-entry tiles per group (register budget)
  constexpr int SW = 16 * NU;           // entries per full group

  __shared__ float g1w[kWaves][kTB][RT];
  __shared__ float g2w[kWaves][kTB][RT];
  __shared__ float g3x[64][RT + 1];  // SW <= 64 rows used
  __shared__ float gsx[kWaves][RT];
  __shared__ float lsx[kWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane & 15, g = lane >> 4;
  const int R = a.R, ns = a.ns, I1 = a.I1, I2 = a.I2, I3 = a.I3;
  const int blk = blockIdx.x * kWaves + wave;
  const bool active = blk < a.nblocks;
  const int b1 = active ? blk / a.nb2 : 0, b2 = active ? blk % a.nb2 : 0;
  const int i10 = b1 * a.tb1, i20 = b2 * a.tb2;
  const int n1 = active ? min(a.tb1, I1 - i10) : 0;
  const int n2 = active ? min(a.tb2, I2 - i20) : 0;
  const bool want_loss = a.want & kWantLoss;

  int jt[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) jt[t] = 16 * (t >> 2) + 4 * g + (t & 3);

  // weights as MFMA operands (zero outside h < ns, j < R)
  auto sval = [&](int h, int j) -> float { return (h < ns && j < R) ? a.S[h][j] : 0.f; };
  float A1op[NH][NT], A2op[NM][NH][4], cv[NH][4];
#pragma unroll
  for (int ht = 0; ht < NH; ++ht) {
#pragma unroll
    for (int t = 0; t < NT; ++t) A1op[ht][t] = sval(16 * ht + n, jt[t]);
#pragma unroll
    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) A2op[mt][ht][t] = sval(16 * ht + 4 * g + t, 16 * mt + n);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int h = 16 * ht + 4 * g + r;
      cv[ht][r] = h < ns ? a.c[h] : 0.f;
    }
  }

  for (int idx = lane; idx < kTB * RT; idx += 64) {
    (&g1w[wave][0][0])[idx] = 0.f;
    (&g2w[wave][0][0])[idx] = 0.f;
  }
  float gsacc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) gsacc[t] = 0.f;
  Kahan<float> lacc;

  const int nfull = I3 / SW;
  const int tail = I3 - SW * nfull;
  const int nsc = nfull + (tail > 0 ? 1 : 0);
  const bool vec = (I3 % NU) == 0;
  const int npairs = n1 * n2;

  for (int sc = 0; sc < nsc; ++sc) {
    const bool wide = sc < nfull;
    const int c0 = SW * sc;
    const int nu = wide ? NU : (tail + 15) >> 4;
    int i3u[NU];
    bool vu[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      i3u[u] = c0 + (wide ? NU * n + u : 16 * u + n);
      vu[u] = u < nu && i3u[u] < I3;
    }
    float a3r[NU][NT], g3[NU][NT];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        a3r[u][t] = (vu[u] && jt[t] < R) ? a.A3[(size_t)i3u[u] * R + jt[t]] : 0.f;
        g3[u][t] = 0.f;
      }

    for (int q = 0; q < npairs; ++q) {
      const int i1l = q / n2, i2l = q - (q / n2) * n2;
      const int i1 = i10 + i1l, i2 = i20 + i2l;
      float W[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        W[t] = jt[t] < R ? a.A1[(size_t)i1 * R + jt[t]] * a.A2[(size_t)i2 * R + jt[t]] : 0.f;
      const size_t base = ((size_t)i1 * I2 + i2) * I3;
      float x[NH][4][NU];
#pragma unroll
      for (int ht = 0; ht < NH; ++ht)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int h = 16 * ht + 4 * g + r;
          if (h < ns) {
            const float* Xh = a.X[h] + base;
            if (wide && vec) {
              if constexpr (NU == 4) {
                const f4 v = *reinterpret_cast<const f4*>(Xh + c0 + 4 * n);
                x[ht][r][0] = v[0];
                x[ht][r][1] = v[1];
                x[ht][r][2] = v[2];
                x[ht][r][3] = v[3];
              } else {
                const f2 v = *reinterpret_cast<const f2*>(Xh + c0 + 2 * n);
                x[ht][r][0] = v[0];
                x[ht][r][1] = v[1];
              }
            } else {
#pragma unroll
              for (int u = 0; u < NU; ++u) x[ht][r][u] = vu[u] ? Xh[i3u[u]] : 0.f;
            }
          } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) x[ht][r][u] = 0.f;
          }
        }

      // GEMM1: model values for 16 h x 16 entries per (h-tile, entry tile)
      f4 D1[NH][NU];
#pragma unroll
      for (int ht = 0; ht < NH; ++ht)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
          if (u < nu) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc = mfma(A1op[ht][t], W[t] * a3r[u][t], acc);
          }
          D1[ht][u] = acc;
        }

      // loss and weighted derivative in place
#pragma unroll
      for (int ht = 0; ht < NH; ++ht)
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float f, y;
            LossFn<float, LOSS>::eval(x[ht][r][u], D1[ht][u][r], f, y);
            const bool ok = vu[u] && cv[ht][r] != 0.f;
            if (want_loss && ok) lacc.add(cv[ht][r] * f);
            D1[ht][u][r] = ok ? cv[ht][r] * y : 0.f;
          }

      // temporal-weight gradient: y_t sits in register 0 of lane group 0
      {
        float ps[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) ps[t] = 0.f;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const float yt = __shfl(D1[0][u][0], n);
#pragma unroll
          for (int t = 0; t < NT; ++t) ps[t] += yt * a3r[u][t];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) gsacc[t] += W[t] * ps[t];
      }

      // GEMM2: yhat[j][e] = sum_h S[h][j] Yc[h][e]
      float Vp[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) Vp[t] = 0.f;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        if (u >= nu) continue;
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ht = 0; ht < NH; ++ht)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(A2op[mt][ht][t], D1[ht][u][t], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int tt = 4 * mt + r;
            g3[u][tt] += acc[r] * W[tt];
            Vp[tt] += acc[r] * a3r[u][tt];
          }
        }
      }
      const float v = row_reduce_scatter<NT>(Vp, n);
      if ((n & ((16 / NT) - 1)) == 0) {
        const int tt = n >> (4 - LOGNT);
        const int j = 16 * (tt >> 2) + 4 * g + (tt & 3);
        if (j < R) {
          g1w[wave][i1l][j] += v * a.A2[(size_t)i2 * R + j];
          g2w[wave][i2l][j] += v * a.A1[(size_t)i1 * R + j];
        }
      }
    }

    // combine the waves' mode-3 rows of this 64-wide group in wave order
    for (int idx = tid; idx < SW * (RT + 1); idx += kThreads) (&g3x[0][0])[idx] = 0.f;
    __syncthreads();
    for (int w = 0; w < kWaves; ++w) {
      if (wave == w) {
#pragma unroll
        for (int u = 0; u < NU; ++u)
          if (vu[u])
#pragma unroll
            for (int t = 0; t < NT; ++t) g3x[i3u[u] - c0][jt[t]] += g3[u][t];
      }
      __syncthreads();
    }
    for (int idx = tid; idx < SW * RT; idx += kThreads) {
      const int l = idx / RT, j = idx - (idx / RT) * RT;
      if (c0 + l < I3 && j < R) a.G3p[((size_t)blockIdx.x * I3 + c0 + l) * R + j] = g3x[l][j];
    }
    __syncthreads();
  }

  // mode-1/2 partial rows of this wave's block
  if (active) {
    for (int idx = lane; idx < kTB * RT; idx += 64) {
      const int l = idx / RT, j = idx - (idx / RT) * RT;
      if (j < R) {
        if (l < n1) a.G1p[((size_t)b2 * I1 + i10 + l) * R + j] = g1w[wave][l][j];
        if (l < n2) a.G2p[((size_t)b1 * I2 + i20 + l) * R + j] = g2w[wave][l][j];
      }
    }
  }
  // temporal-weight gradient and objective partials of the workgroup
  {
    float gv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) gv[t] = gsacc[t];
    // sum over the 16 lanes of the row, then over the 4 rows
    const float v = row_reduce_scatter<NT>(gv, n);
    float vs = v;
    if ((n & ((16 / NT) - 1)) == 0) {
      const int tt = n >> (4 - LOGNT);
      gsx[wave][16 * (tt >> 2) + 4 * g + (tt & 3)] = vs;
    }
    float ls = lacc.s;
    for (int m = 32; m >= 1; m >>= 1) ls += __shfl_xor(ls, m);
    if (lane == 0) lsx[wave] = ls;
  }
  __syncthreads();
  if (tid < R) {
    float s = 0.f;
    for (int w = 0; w < kWaves; ++w) s += gsx[w][tid];
    a.gsp[(size_t)blockIdx.x * R + tid] = s;
  }
  if (tid == 0) {
    float s = 0.f;
    for (int w = 0; w < kWaves; ++w) s += lsx[w];
    a.lossp[blockIdx.x] = s;
  }
}

template <int LOSS, int RT, int NH>
hipError_t launch(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p, float* gsp,
                  float* lossp) {
  MArgs a;
  for (int h = 0; h < c.ns; ++h) {
    a.X[h] = static_cast<const float*>(c.X[h]);
    a.S[h] = static_cast<const float*>(c.S[h]);
    a.c[h] = (float)c.c[h];
  }
  a.A1 = static_cast<const float*>(c.A[0]);
  a.A2 = static_cast<const float*>(c.A[1]);
  a.A3 = static_cast<const float*>(c.A[2]);
  a.G1p = G1p;
  a.G2p = G2p;
  a.G3p = G3p;
  a.gsp = gsp;
  a.lossp = lossp;
  a.I1 = c.I1; a.I2 = c.I2; a.I3 = c.I3; a.R = c.R; a.ns = c.ns; a.want = c.want;
  a.tb1 = p.tb1; a.tb2 = p.tb2; a.nb2 = p.nb2; a.nblocks = p.nblocks;
  hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, NH>), dim3(p.nwg), dim3(kThreads), 0, c.stream, a);
  return hipGetLastError();
}

template <int LOSS, int RT>
hipError_t by_nh(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p, float* gsp,
                 float* lossp) {
  if (c.ns <= 16) return launch<LOSS, RT, 1>(c, p, G1p, G2p, G3p, gsp, lossp);
  if (c.ns <= 32) return launch<LOSS, RT, 2>(c, p, G1p, G2p, G3p, gsp, lossp);
  if (c.ns <= 48) return launch<LOSS, RT, 3>(c, p, G1p, G2p, G3p, gsp, lossp);
  return launch<LOSS, RT, 4>(c, p, G1p, G2p, G3p, gsp, lossp);
}

template <int LOSS>
hipError_t by_rank(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p, float* gsp,
                   float* lossp) {
  if (c.R <= 16) return by_nh<LOSS, 16>(c, p, G1p, G2p, G3p, gsp, lossp);
  return by_nh<LOSS, 32>(c, p, G1p, G2p, G3p, gsp, lossp);
}

}  // namespace

bool mfma_supported(int R, int ns, int dtype) { return dtype == 0 && R >= 1 && R <= 32 && ns <= 64; }

MfmaPlan mfma_plan(int I1, int I2, int I3) {
  (void)I3;
  MfmaPlan p;
  const long pairs = (long)I1 * I2;
  const long target_blocks = 4096;
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
    case kGaussian: return by_rank<kGaussian>(c, p, G1p, G2p, G3p, gsp, lossp);
    case kPoissonLog: return by_rank<kPoissonLog>(c, p, G1p, G2p, G3p, gsp, lossp);
    default: return by_rank<kBernoulliLogit>(c, p, G1p, G2p, G3p, gsp, lossp);
  }
}

}  // namespace gcp
