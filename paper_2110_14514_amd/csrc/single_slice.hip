// Objective and gradients over ONE dense slice (no stored window), with the
// three rank contractions on the FP32 matrix cores.
//
// With a single slice the window kernel's slice rows (GEMM1's M dimension)
// would hold one useful row in sixteen.  Here the sixteen rows are sixteen
// (i1, i2) pairs instead: a wave owns a 4 x 4 block of pairs, p = 4a + b for
// (i1, i2) = (i10 + a, i20 + b), and walks I3 in groups of 32 entries (two
// 16-entry tiles u, entry c0 + 2c + u in column c).  Per tile:
//   GEMM1  m[p][c]  = sum_j (s_j A1[i1,j] A2[i2,j]) A3[e(c),j]          (K = j)
//   loss   f, y = df/dm                                                   (VALU)
//   GEMM2  G3[j][c] += sum_p (s_j A1[i1,j] A2[i2,j]) y[p][c]            (K = p)
//   GEMM3  V[j][p]  += sum_c A3[e(c),j] y[p][c]                          (K = c)
// GEMM1's accumulator (rows p, columns c) is GEMM2's B operand as it sits in
// the registers; GEMM3 needs y with the entries along K, so the tile goes
// through a per-wave LDS transpose.  V accumulates over the whole I3 walk;
// at the end of the block
//   G1[i1,j] += s_j sum_b A2[i2_b,j] V[4a+b][j]   (a quad of lanes)
//   G2[i2,j] += s_j sum_a A1[i1_a,j] V[4a+b][j]   (lanes 4 apart)
//   g_s[j]   += sum_p A1[i1,j] A2[i2,j] V[p][j]   (the 16 lanes of a row)
// (eqs. gcp_grad_A / gcp_grad_lambda of Section 4.2 with the window empty),
// so no per-entry vector work is left but the loss.  G3 rows of a group are
// combined over the workgroup's waves in a fixed order; every partial goes to
// a block- or workgroup-indexed slot that the fixed-order reduce sums, so the
// results are bitwise reproducible.
#include "mfma_tile.hpp"

namespace gcp {
namespace {

constexpr int kSsPitch = 20;   // padded LDS row (16-byte reads of 16 lanes hit every bank once)
constexpr int kSsWaves = 4;    // pair blocks (waves) per workgroup
constexpr int kSsThreads = 64 * kSsWaves;

struct SsArgs {
  const float* X;
  const float* s;
  const float* A1;
  const float* A2;
  const float* A3;
  float* G1p;
  float* G2p;
  float* G3p;
  float* gsp;
  float* lossp;
  int I1, I2, I3, R, nb1, nb2, nblocks;
  int xbits;        // X bit-packed: rows of rpw 32-bit words, entry i3 = bit i3 % 32 of word i3 / 32
  int rpw;
};

// A3 rows of one group of 32 entries in the two layouts the tile reads
__host__ __device__ constexpr int ss_a3_floats(int RT) { return 2 * RT * kSsPitch + 2 * 16 * (RT + 4); }

__host__ __device__ constexpr int ss_lds_floats(int RT) {
  return 2 * ss_a3_floats(RT)               // A3 of a group, two buffers
         + kSsWaves * 2 * 16 * kSsPitch     // per-wave y transposes [u][p][c]
         + 2 * kSsWaves * 32 * RT           // per-wave G3 rows of a group, two buffers
         + kSsWaves * RT + kSsWaves;        // per-wave g_s and objective
}

template <int LOSS, int RT, bool XB>
__global__ void __launch_bounds__(kSsThreads) __attribute__((amdgpu_waves_per_eu(RT == 16 ? 4 : 2, 4)))
single_slice_kernel(SsArgs a) {
  constexpr int NT = RT / 4;    // GEMM1 K steps
  constexpr int NM = RT / 16;   // 16-column tiles of j
  constexpr int NA = 32 * RT / kSsThreads;   // A3 values a thread stages per group
  static_assert(NA * kSsThreads == 32 * RT, "a group's A3 values split evenly over the threads");
  __shared__ __attribute__((aligned(16))) float lds[ss_lds_floats(RT)];
  float* a3buf = lds;                                      // [buf]{[u][j][c], [u][c][j]}
  float* ytr_all = a3buf + 2 * ss_a3_floats(RT);           // [wave][u][p][c]
  float* g3w_all = ytr_all + kSsWaves * 2 * 16 * kSsPitch; // [buf][wave][e][j]
  float* gsw = g3w_all + 2 * kSsWaves * 32 * RT;
  float* lsw = gsw + kSsWaves * RT;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 15, g = lane >> 4;
  float* ytr = ytr_all + wave * 2 * 16 * kSsPitch;
  const int R = a.R, I1 = a.I1, I2 = a.I2, I3 = a.I3;
  const int blk = blockIdx.x * kSsWaves + wave;
  const bool active = blk < a.nblocks;
  const int b1 = active ? blk / a.nb2 : 0, b2 = active ? blk % a.nb2 : 0;
  const int i10 = 4 * b1, i20 = 4 * b2;
  const int n1 = active ? min(4, I1 - i10) : 0, n2 = active ? min(4, I2 - i20) : 0;
  auto pvalid = [&](int p) { return (p >> 2) < n1 && (p & 3) < n2; };
  auto pair_i1 = [&](int p) { return pvalid(p) ? i10 + (p >> 2) : 0; };
  auto pair_i2 = [&](int p) { return pvalid(p) ? i20 + (p & 3) : 0; };

  // GEMM1 A operand: row n = pair p, K step t <-> j = 16 (t/4) + 4g + t%4
  float S1[NT];
  {
    const bool v = pvalid(n);
    const float* r1 = a.A1 + (size_t)pair_i1(n) * R;
    const float* r2 = a.A2 + (size_t)pair_i2(n) * R;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int j = 16 * (t >> 2) + 4 * g + (t & 3);
      const int jc = min(j, R - 1);
      S1[t] = (v && j < R) ? MLoss<LOSS>::kM * a.s[jc] * r1[jc] * r2[jc] : 0.f;
    }
  }
  // GEMM2 A operand: row n <-> j = 16 mt + n, K step t <-> pair p = 4g + t
  float C2[NM][4];
#pragma unroll
  for (int mt = 0; mt < NM; ++mt)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int p = 4 * g + t, j = 16 * mt + n, jc = min(j, R - 1);
      C2[mt][t] = (pvalid(p) && j < R)
                      ? MLoss<LOSS>::kY * a.s[jc] * a.A1[(size_t)pair_i1(p) * R + jc] * a.A2[(size_t)pair_i2(p) * R + jc]
                      : 0.f;
    }
  // rows of X held by this lane: pair p = 4g + r
  size_t xrow[4];
  bool rv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = 4 * g + r;
    rv[r] = pvalid(p);
    xrow[r] = ((size_t)pair_i1(p) * I2 + pair_i2(p)) * I3;
  }
  // this lane's slice values of group sc: pair 4g + r, entries 32 sc + 2n + u.
  // Loads are unconditional: a pair past the slice reads row 0 and an entry
  // past the row reads the row's last value.  Those terms never count: their
  // GEMM1/GEMM2 operand rows (pairs) or A3 rows (entries) are zero and their
  // objective terms are masked.
  const float* xr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    xr[r] = XB ? a.X + ((size_t)pair_i1(4 * g + r) * I2 + pair_i2(4 * g + r)) * a.rpw : a.X + xrow[r];
  // Bit-packed slices: the raw word of group sc is held (its bits 2n + u
  // are the lane's entries) and unpacked where the values are used.
  auto load_x = [&](int sc, float (&xv)[4][2]) {
    const int c0 = 32 * sc;
    if constexpr (XB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) xv[r][0] = xr[r][sc];
    } else {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = min(c0 + 2 * n + u, I3 - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[r][u] = xr[r][e];
      }
    }
  };
  auto xval = [&](const float (&xv)[4][2], int r, int u) -> float {
    if constexpr (XB) return (float)((__float_as_uint(xv[r][0]) >> (2 * n + u)) & 1u);
    return xv[r][u];
  };
  // the group's A3 values, thread value k <-> (u, c, j) with j fastest so
  // that the lanes read whole A3 rows (zero past the row and past R)
  auto load_a3 = [&](int sc, float (&av)[NA]) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int idx = tid + k * kSsThreads;
      const int j = idx % RT, c = (idx / RT) % 16, u = idx / (16 * RT);
      const int e = 32 * sc + 2 * c + u;
      av[k] = (e < I3 && j < R) ? a.A3[(size_t)e * R + j] : 0.f;
    }
  };
  auto store_a3 = [&](int buf, const float (&av)[NA]) {
    float* a3t = a3buf + buf * ss_a3_floats(RT);
    float* a3g = a3t + 2 * RT * kSsPitch;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int idx = tid + k * kSsThreads;
      const int j = idx % RT, c = (idx / RT) % 16, u = idx / (16 * RT);
      a3t[(u * RT + j) * kSsPitch + c] = av[k];
      a3g[(u * 16 + c) * (RT + 4) + j] = av[k];
    }
  };

  // V of the even and the odd 16-entry tiles kept apart, so that the two
  // tiles' matrix-core chains of a group are independent and interleave
  f4 V2[2][NM];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int mt = 0; mt < NM; ++mt) V2[u][mt] = f4{0.f, 0.f, 0.f, 0.f};
  Kahan<float> lacc;
  const int ngroups = (I3 + 31) / 32;
  // software pipeline: the slice values and A3 rows of group sc + 1 are in
  // flight while group sc computes; A3 and the per-wave G3 rows alternate
  // between two LDS buffers, so one barrier per group separates
  //   [compute sc, write G3 rows (buf sc), stage A3 of sc + 1 (buf sc + 1)]
  // from [combine the G3 rows of sc, compute sc + 1].
  float xc[4][2], xn[4][2];
  float an[NA];
  load_x(0, xc);
  load_a3(0, an);
  store_a3(0, an);
  __syncthreads();
  for (int sc = 0; sc < ngroups; ++sc) {
    const int c0 = 32 * sc, buf = sc & 1;
    const bool more = sc + 1 < ngroups;
    if (more) {
      load_x(sc + 1, xn);
      load_a3(sc + 1, an);
    }
    const float* a3t = a3buf + buf * ss_a3_floats(RT);
    const float* a3g = a3t + 2 * RT * kSsPitch;
    bool ev[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) ev[u] = c0 + 2 * n + u < I3;
    f4 G3acc[2][NM];
    float fgroup = 0.f;   // the group's objective terms (compensated once per group)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // GEMM1 B operand: column n of tile u, K step t <-> j = 16 (t/4) + 4g + t%4
      float B1[NT];
#pragma unroll
      for (int t4 = 0; t4 < NT / 4; ++t4) {
        const f4 v = *reinterpret_cast<const f4*>(a3g + (u * 16 + n) * (RT + 4) + 16 * t4 + 4 * g);
#pragma unroll
        for (int r = 0; r < 4; ++r) B1[4 * t4 + r] = v[r];
      }
      f4 D = {0.f, 0.f, 0.f, 0.f};
      if constexpr (LOSS != kGaussianId) {
#pragma unroll
        for (int t = 0; t < NT; ++t) D = mfma(S1[t], B1[t], D);
      }
      // loss derivative in place; objective terms of valid (pair, entry)
      float fpart = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float f = 0.f;
        D[r] = MLoss<LOSS>::fy(xval(xc, r, u), D[r], 1.f, f);
        fpart += (rv[r] && ev[u]) ? f : 0.f;
      }
      fgroup += fpart;
      // GEMM2: G3[j][c] over the block's pairs
#pragma unroll
      for (int mt = 0; mt < NM; ++mt) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = mfma(C2[mt][t], D[t], acc);
        G3acc[u][mt] = acc;
      }
      // y tile transposed through this wave's LDS: row p, column c
      float* yt = ytr + u * 16 * kSsPitch;
#pragma unroll
      for (int r = 0; r < 4; ++r) yt[(4 * g + r) * kSsPitch + n] = D[r];
      // the wave's LDS operations complete in order; keep the compiler from
      // moving the read above the other lanes' writes
      __builtin_amdgcn_wave_barrier();
      const f4 yv = *reinterpret_cast<const f4*>(yt + n * kSsPitch + 4 * g);
      __builtin_amdgcn_wave_barrier();
      // GEMM3: V[j][p] += sum_c A3[e(c)][j] y[p][c], K step t <-> c = 4g + t
#pragma unroll
      for (int mt = 0; mt < NM; ++mt) {
        const f4 av = *reinterpret_cast<const f4*>(a3t + (u * RT + 16 * mt + n) * kSsPitch + 4 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t) V2[u][mt] = mfma(av[t], yv[t], V2[u][mt]);
      }
    }
    lacc.add(fgroup);
    // G3 rows of the group: each wave's block into buffer buf
    float* g3w = g3w_all + (buf * kSsWaves + wave) * 32 * RT;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) g3w[(2 * n + u) * RT + 16 * mt + 4 * g + r] = G3acc[u][mt][r];
    if (more) store_a3(buf ^ 1, an);
    __syncthreads();
    // the waves' G3 rows summed in a fixed order
    const float* g3b = g3w_all + buf * kSsWaves * 32 * RT;
    for (int idx = tid; idx < 32 * RT; idx += kSsThreads) {
      const int e = idx / RT, j = idx - (idx / RT) * RT;
      if (c0 + e < I3 && j < R) {
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < kSsWaves; ++w) sum += g3b[w * 32 * RT + idx];
        a.G3p[((size_t)blockIdx.x * I3 + c0 + e) * R + j] = sum;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int u = 0; u < 2; ++u) xc[r][u] = xn[r][u];
  }

  // V[j][p] of this lane: j = 16 mt + 4g + r, p = n.  Mode-1/2 rows and the
  // temporal gradient of the block.
  f4 V[NM];
#pragma unroll
  for (int mt = 0; mt < NM; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) V[mt][r] = V2[0][mt][r] + V2[1][mt][r];
  {
    const int p = n;
    const bool v = pvalid(p);
    const float* r1 = a.A1 + (size_t)pair_i1(p) * R;
    const float* r2 = a.A2 + (size_t)pair_i2(p) * R;
    float gsv[NM][4];
#pragma unroll
    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * mt + 4 * g + r, jc = min(j, R - 1);
        const bool ok = v && j < R;
        const float a1 = ok ? r1[jc] : 0.f, a2 = ok ? r2[jc] : 0.f, sj = j < R ? a.s[jc] : 0.f;
        const float vv = V[mt][r];
        // G1 row i1 = i10 + a: sum over b (the four lanes of a quad)
        float t1 = vv * a2;
        t1 += row_xor1(t1);
        t1 += row_xor2(t1);
        // G2 row i2 = i20 + b: sum over a (lanes 4 apart)
        float t2 = vv * a1;
        t2 += row_xor4(t2);
        t2 += row_xor8(t2);
        // g_s: sum over the 16 pairs
        float t3 = vv * a1 * a2;
        t3 += row_xor1(t3);
        t3 += row_xor2(t3);
        t3 += row_xor4(t3);
        t3 += row_xor8(t3);
        gsv[mt][r] = t3;
        if (active && j < R) {
          if ((p & 3) == 0 && (p >> 2) < n1)
            a.G1p[((size_t)b2 * I1 + i10 + (p >> 2)) * R + j] = MLoss<LOSS>::kY * sj * t1;
          if ((p >> 2) == 0 && (p & 3) < n2)
            a.G2p[((size_t)b1 * I2 + i20 + (p & 3)) * R + j] = MLoss<LOSS>::kY * sj * t2;
        }
      }
    if (n == 0) {
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) gsw[wave * RT + 16 * mt + 4 * g + r] = MLoss<LOSS>::kY * gsv[mt][r];
    }
    float ls = MLoss<LOSS>::kF * lacc.s;
    for (int m = 32; m >= 1; m >>= 1) ls += __shfl_xor(ls, m);
    if (lane == 0) lsw[wave] = ls;
  }
  __syncthreads();
  if (tid < R) {
    float sum = 0.f;
    for (int w = 0; w < kSsWaves; ++w) sum += gsw[w * RT + tid];
    a.gsp[(size_t)blockIdx.x * R + tid] = sum;
  }
  if (tid == 0) {
    float sum = 0.f;
    for (int w = 0; w < kSsWaves; ++w) sum += lsw[w];
    a.lossp[blockIdx.x] = sum;
  }
}

template <int LOSS>
hipError_t ss_launch_rt(const DenseCall& c, const SsArgs& a, int nwg) {
  if constexpr (LOSS == kBernoulliLogit || LOSS == kBernoulliOdds) {
    if (c.xbits) {
      if (c.R <= 16)
        hipLaunchKernelGGL((single_slice_kernel<LOSS, 16, true>), dim3(nwg), dim3(kSsThreads), 0, c.stream, a);
      else
        hipLaunchKernelGGL((single_slice_kernel<LOSS, 32, true>), dim3(nwg), dim3(kSsThreads), 0, c.stream, a);
      return hipGetLastError();
    }
  }
  if (c.xbits) return hipErrorInvalidValue;   // bit-packed slices are binary data
  if (c.R <= 16)
    hipLaunchKernelGGL((single_slice_kernel<LOSS, 16, false>), dim3(nwg), dim3(kSsThreads), 0, c.stream, a);
  else
    hipLaunchKernelGGL((single_slice_kernel<LOSS, 32, false>), dim3(nwg), dim3(kSsThreads), 0, c.stream, a);
  return hipGetLastError();
}

}  // namespace

SsPlan single_slice_plan(int I1, int I2) {
  SsPlan p;
  p.nb1 = (I1 + 3) / 4;
  p.nb2 = (I2 + 3) / 4;
  p.nblocks = p.nb1 * p.nb2;
  p.nwg = (p.nblocks + kSsWaves - 1) / kSsWaves;
  return p;
}

bool single_slice_supported(const DenseCall& c) {
  return c.ns == 1 && c.dtype == 0 && c.R >= 1 && c.R <= 32 && c.kernel != 1 && c.loss <= kBernoulliOdds;
}

hipError_t single_slice_launch(const DenseCall& c, float* G1p, float* G2p, float* G3p, float* gsp, float* lossp) {
  const SsPlan pl = single_slice_plan(c.I1, c.I2);
  SsArgs a;
  a.X = static_cast<const float*>(c.X[0]);
  a.s = static_cast<const float*>(c.S[0]);
  a.A1 = static_cast<const float*>(c.A[0]);
  a.A2 = static_cast<const float*>(c.A[1]);
  a.A3 = static_cast<const float*>(c.A[2]);
  a.G1p = G1p;
  a.G2p = G2p;
  a.G3p = G3p;
  a.gsp = gsp;
  a.lossp = lossp;
  a.I1 = c.I1; a.I2 = c.I2; a.I3 = c.I3; a.R = c.R;
  a.nb1 = pl.nb1; a.nb2 = pl.nb2; a.nblocks = pl.nblocks;
  a.xbits = c.xbits;
  a.rpw = (c.I3 + 31) / 32;
  switch (c.loss) {
    case kGaussian: return ss_launch_rt<kGaussian>(c, a, pl.nwg);
    case kPoissonLog: return ss_launch_rt<kPoissonLog>(c, a, pl.nwg);
    case kBernoulliLogit: return ss_launch_rt<kBernoulliLogit>(c, a, pl.nwg);
    case kGaussianId: return ss_launch_rt<kGaussianId>(c, a, pl.nwg);
    case kPoissonId: return ss_launch_rt<kPoissonId>(c, a, pl.nwg);
    default: return ss_launch_rt<kBernoulliOdds>(c, a, pl.nwg);
  }
}

}  // namespace gcp
