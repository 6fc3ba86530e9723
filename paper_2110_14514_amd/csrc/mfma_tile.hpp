// Fused objective/gradient over a dense slice and its window, with the two
// rank-R contractions on the FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Same quantities as the VALU kernel (eq. gcp_stream_problem_1 and the
// gradients of Section 4.2), organised around two small GEMMs per group of
// 64 entries e of one (i1,i2) pair row:
//   GEMM1  m[h][e]  = sum_j S[h][j] P[e][j],  P[e][j] = A1[i1,j] A2[i2,j] A3[i3,j]
//   GEMM2  yhat[j][e] = sum_h (c_h S[h][j]) y(x_he, m[h][e])
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
// Entries: a full group is NU = 2 16-column tiles u (32 entries, sized to the
// register file) with i3 = c0 + 2n + u, so each lane loads 2 contiguous
// values per slice; the ragged tail of a row uses i3 = c0 + 16u + n with only
// the tiles that hold entries.
//
// Work decomposition: each wave owns a TB1 x TB2 block of pairs over all of
// I3; eight waves form a workgroup that combines its waves' mode-3 rows and
// temporal-gradient partials in a fixed order.  All partials go to
// block/workgroup-indexed slots and are summed in a fixed order by the
// reduce kernel, so results are bitwise reproducible.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace gcp {
namespace {


typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = kBatchTileWaves;   // rank tile 16 and the batched builds
constexpr int kThreads = 64 * kWaves;
constexpr int kTB = 16;
// waves per workgroup of a single stream's build at rank tile RT
__host__ __device__ constexpr int tile_waves(int RT) { return single_tile_waves(RT); }
// Minimum waves per SIMD a single stream's build is compiled for (its
// register budget): 3 (168 registers) for rank tile 32 with one h-tile, one
// pair per step and 16-byte copies, which fit so without spills in the pair
// loop (its 54.5 KB of LDS, rounded up to the allocation granule, still
// admits two workgroups per compute unit); 2 (256 registers) otherwise.
template <int RT, int NH, int PK, int DMA16>
constexpr int tile_min_waves() { return RT == 32 && NH == 1 && PK == 1 && DMA16 != 0 ? 3 : 2; }

// Everything one workgroup needs for its tile of pair blocks.  Slice h = 0 is
// the current slice; slice h >= 1 is window slot h-1 of the ring (slot order),
// with weight row s_{h} at shist + (h-1) R.
struct TileArgs {
  const float* Xt;
  const float* ring;
  size_t rstride;   // elements per stored slice
  size_t rp3;       // row pitch of stored slices (X_t rows have pitch I3)
  const float* st;
  const float* shist;
  const float* A1;
  const float* A2;
  const float* A3;
  float* G1p;
  float* G2p;
  float* G3p;
  float* gsp;
  float* lossp;
  int I1, I2, I3, R, ns, want, tb1, tb2, nb2, nblocks;
  int nch, gpc;     // I3 chunks of the launch, 32-entry groups per chunk
  int rpw;          // bit-packed slices: 32-bit words per (i1, i2) row
};

struct MArgs {
  TileArgs t;
  float c[kMaxNs];
};

// Per-wave LDS ring of the staged pipeline: kStages stages, each holding
// 16*NH slice rows of 32 values and the pair's two factor rows (64 values:
// A1 row at 0, A2 row at 32).  With two pairs per stage (PK = 2) pair B's
// rows sit at pair_b_offset: in the unused upper halves (16, 48) at rank
// tile 16, after pair A's (64, 96) at rank tile 32.  XS (16-byte copies of
// the stored rows): row i holds stored slice i + 1, and the last row of the
// pair's rows (16 NH - 1, or 8p + 7 with PK = 2), whose slice is always past
// the window, holds the current slice, copied 4 bytes at a time because its
// start need not be 16-byte aligned.
constexpr int kStages = 3;
__host__ __device__ constexpr int pair_b_offset(int RT) { return RT > 16 ? 64 : 16; }
__host__ __device__ constexpr int stage_floats(int NH, int PK = 1, int RT = 16) {
  return 16 * NH * 32 + (PK == 2 && RT > 16 ? 128 : 64);
}
__host__ __device__ constexpr int ring_floats(int NH, int PK, int RT, int WV) {
  return NH <= 2 ? WV * kStages * stage_floats(NH, PK, RT) : 0;
}

// LDS floats used by one workgroup at rank tile RT and NH h-tiles: the
// mode-3 combine rows (NH > 2; with NH <= 2 the idle staging rings serve),
// the temporal-gradient rows and the objective partials of the waves
__host__ __device__ constexpr int lds_floats(int RT, int NH, int WV) {
  return (NH > 2 ? 64 * (RT + 1) : 0) + WV * (RT + 1);
}
__host__ __device__ constexpr int lds_gs_offset(int RT, int NH) { return NH > 2 ? 64 * (RT + 1) : 0; }
// The group's A3 values in GEMM2's transposed output layout, shared by the
// workgroup's waves: [tile u][column j][row 4g + r], rows padded to 20
// floats so that a 16-byte read by the 16 lanes of a row group touches
// every bank once.
constexpr int kA3TPitch = 20;
// ... and in GEMM1's operand layout: [tile u][column n][j], rows padded to
// RT + 4 floats for the same reason.
__host__ __device__ constexpr int a3g_pitch(int RT) { return RT + 4; }
__host__ __device__ constexpr int a3t_floats(int RT) { return 2 * RT * kA3TPitch + 2 * 16 * a3g_pitch(RT); }

// Wait until at most n vector-memory operations of this wave are in flight
// (n is wave-uniform; the immediate must be a constant).  n >= 40 waits for
// 40, which is always safe (it only waits longer).
__device__ __forceinline__ void wait_vmcnt(int n) {
#if defined(__HIP_DEVICE_COMPILE__)
  switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
    case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
    case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    case 9: asm volatile("s_waitcnt vmcnt(9)" ::: "memory"); break;
    case 10: asm volatile("s_waitcnt vmcnt(10)" ::: "memory"); break;
    case 11: asm volatile("s_waitcnt vmcnt(11)" ::: "memory"); break;
    case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
    case 13: asm volatile("s_waitcnt vmcnt(13)" ::: "memory"); break;
    case 14: asm volatile("s_waitcnt vmcnt(14)" ::: "memory"); break;
    case 15: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
    case 16: asm volatile("s_waitcnt vmcnt(16)" ::: "memory"); break;
    case 17: asm volatile("s_waitcnt vmcnt(17)" ::: "memory"); break;
    case 18: asm volatile("s_waitcnt vmcnt(18)" ::: "memory"); break;
    case 19: asm volatile("s_waitcnt vmcnt(19)" ::: "memory"); break;
    case 20: asm volatile("s_waitcnt vmcnt(20)" ::: "memory"); break;
    case 21: asm volatile("s_waitcnt vmcnt(21)" ::: "memory"); break;
    case 22: asm volatile("s_waitcnt vmcnt(22)" ::: "memory"); break;
    case 23: asm volatile("s_waitcnt vmcnt(23)" ::: "memory"); break;
    case 24: asm volatile("s_waitcnt vmcnt(24)" ::: "memory"); break;
    case 25: asm volatile("s_waitcnt vmcnt(25)" ::: "memory"); break;
    case 26: asm volatile("s_waitcnt vmcnt(26)" ::: "memory"); break;
    case 27: asm volatile("s_waitcnt vmcnt(27)" ::: "memory"); break;
    case 28: asm volatile("s_waitcnt vmcnt(28)" ::: "memory"); break;
    case 29: asm volatile("s_waitcnt vmcnt(29)" ::: "memory"); break;
    case 30: asm volatile("s_waitcnt vmcnt(30)" ::: "memory"); break;
    case 31: asm volatile("s_waitcnt vmcnt(31)" ::: "memory"); break;
    case 32: asm volatile("s_waitcnt vmcnt(32)" ::: "memory"); break;
    case 33: asm volatile("s_waitcnt vmcnt(33)" ::: "memory"); break;
    case 34: asm volatile("s_waitcnt vmcnt(34)" ::: "memory"); break;
    case 35: asm volatile("s_waitcnt vmcnt(35)" ::: "memory"); break;
    case 36: asm volatile("s_waitcnt vmcnt(36)" ::: "memory"); break;
    case 37: asm volatile("s_waitcnt vmcnt(37)" ::: "memory"); break;
    case 38: asm volatile("s_waitcnt vmcnt(38)" ::: "memory"); break;
    case 39: asm volatile("s_waitcnt vmcnt(39)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(40)" ::: "memory"); break;
  }
#else
  (void)n;
#endif
}

// A row of zeros: the source of staged rows past the window.
__device__ __attribute__((aligned(16))) float g_zero_row[32];

// Direct global -> LDS copy of `bytes` (4 or 16) per lane: lane i writes at
// lds + i * bytes (lds is wave-uniform); completion is counted by vmcnt.
__device__ __forceinline__ void load_to_lds(const float* src, float* lds, int bytes) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (bytes == 16)
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
#else
  (void)src; (void)lds; (void)bytes;
#endif
}



__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Bitwise select that cannot be turned into a select of addresses (which
// would force the array it reads from into private memory).
__device__ __forceinline__ float pick(bool c, float a, float b) {
  const unsigned m = 0u - (unsigned)c;
  return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
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
      const float lo_v = v[i], hi_v = v[i + half];
      const float send = pick(hi, lo_v, hi_v);
      const float keep = pick(hi, hi_v, lo_v);
      v[i] = keep + __shfl_xor(send, mask);
    }
    mask >>= 1;
  }
  float r = v[0];
  for (; mask >= 1; mask >>= 1) r += __shfl_xor(r, mask);
  return r;
}

// Fire-and-forget LDS add.  Issued as an instruction the compiler does not
// model: an LDS atomic it sees is treated as possibly aliasing the in-flight
// direct-to-LDS copies and would be preceded by a wait for all of them.
// Callers only target LDS arrays that no copy writes, and read them back
// after a barrier; LDS operations complete in order, so the compiler's own
// lgkmcnt waits stay conservative.
__device__ __forceinline__ void lds_add(float* p, float v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned off = (unsigned)(size_t)(__attribute__((address_space(3))) float*)p;
  asm volatile("ds_add_f32 %0, %1" ::"v"(off), "v"(v) : "memory");
#else
  (void)p; (void)v;
#endif
}

// Lane exchanges inside a 16-lane row on the VALU (DPP), no LDS round trip:
// xor 8 is a rotation of the row by 8; xor 4 is the half-row mirror (lane
// i <- 7 - i in each 8-lane half, i.e. xor 7) followed by the quad
// permutation [3,2,1,0] (xor 3); xor 2 and xor 1 are quad permutations.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float row_xor8(float v) { return dpp<0x128>(v); }
__device__ __forceinline__ float row_xor4(float v) { return dpp<0x1B>(dpp<0x141>(v)); }
__device__ __forceinline__ float row_xor2(float v) { return dpp<0x4E>(v); }
__device__ __forceinline__ float row_xor1(float v) { return dpp<0xB1>(v); }

template <int M>
__device__ __forceinline__ float row_xor(float v) {
  if constexpr (M == 8) return row_xor8(v);
  else if constexpr (M == 4) return row_xor4(v);
  else if constexpr (M == 2) return row_xor2(v);
  else return row_xor1(v);
}

// One reduce-scatter step over lane bit M: the lane keeps the upper half of
// its H values when the bit is set, and adds the partner's copy of that half.
template <int M, int H, int NT>
__device__ __forceinline__ void rs_step(float (&v)[NT], int n) {
  const bool hi = (n & M) != 0;
#pragma unroll
  for (int i = 0; i < H / 2; ++i) {
    const float lo_v = v[i], hi_v = v[i + H / 2];
    v[i] = pick(hi, hi_v, lo_v) + row_xor<M>(pick(hi, lo_v, hi_v));
  }
}

// Sum of a value over the four 16-lane groups (lanes n, n+16, n+32, n+48),
// left in every lane: a swap of the wave's halves, then of odd and even
// lane groups (gfx950 lane-swap instructions), each followed by an add.
// Every lane forms (v_n + v_n+32) + (v_n+16 + v_n+48).
__device__ __forceinline__ float sum_lane_groups(float v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const float a = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(a), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
#else
  return v;
#endif
}

// Same result and lane mapping as row_reduce_scatter, with DPP exchanges.
template <int NT>
__device__ __forceinline__ float row_reduce_scatter_dpp(float (&v)[NT], int n) {
  static_assert(NT == 4 || NT == 8, "rank tile of 16 or 32");
  rs_step<8, NT>(v, n);
  rs_step<4, NT / 2>(v, n);
  if constexpr (NT == 8) {
    rs_step<2, 2>(v, n);
    return v[0] + row_xor1(v[0]);
  } else {
    float r = v[0] + row_xor2(v[0]);
    return r + row_xor1(r);
  }
}

// Loss terms in the form the matrix-core kernel evaluates them.  GEMM1's
// operand carries kM, so it returns d = kM m (kM = log2 e for the exponential
// losses: exp(m) is then a single exp2); GEMM2's operand and the temporal
// gradient carry kY (2 for the Gaussian loss, whose y = 2 (m - x)), so the
// per-entry derivative formed here is y / kY; and the objective terms formed
// here are f / kF, the lane sums being scaled by kF once at the end.  fy adds
// cv f / kF to facc and returns y / kY.
template <int LOSS>
struct MLoss;

template <>
struct MLoss<kGaussian> {
  static constexpr float kM = 1.f, kY = 2.f, kF = 1.f;
  __device__ __forceinline__ static float y(float x, float d) { return d - x; }
  __device__ __forceinline__ static float fy(float x, float d, float cv, float& facc) {
    const float yv = d - x;
    facc = fmaf(cv * yv, yv, facc);   // (m - x)^2
    return yv;
  }
  __device__ __forceinline__ static float fr(float x, float d, float& facc) {
    const float yv = d - x;
    facc = fmaf(yv, yv, facc);
    return yv;
  }
};

template <>
struct MLoss<kPoissonLog> {
  static constexpr float kM = 1.44269504088896341f, kY = 1.f, kF = 0.693147180559945309f;
  __device__ __forceinline__ static float y(float x, float d) { return __builtin_amdgcn_exp2f(d) - x; }
  __device__ __forceinline__ static float fy(float x, float d, float cv, float& facc) {
    const float e = __builtin_amdgcn_exp2f(d);
    facc = fmaf(cv, fmaf(-x, d, e * kM), facc);   // (exp(m) - x m) / ln 2
    return e - x;
  }
  __device__ __forceinline__ static float fr(float x, float d, float& facc) {
    const float e = __builtin_amdgcn_exp2f(d);
    facc = fmaf(e, kM, fmaf(-x, d, facc));
    return e - x;
  }
};

template <>
struct MLoss<kBernoulliLogit> {
  static constexpr float kM = 1.44269504088896341f, kY = 1.f, kF = 0.693147180559945309f;
  __device__ __forceinline__ static float y(float x, float d) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(d));
    const float inv = __builtin_amdgcn_rcpf(1.f + e);
    return (d >= 0.f ? inv : e * inv) - x;
  }
  __device__ __forceinline__ static float fy(float x, float d, float cv, float& facc) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(d));
    const float inv = __builtin_amdgcn_rcpf(1.f + e);
    // (max(m, 0) + log(1 + exp(-|m|)) - x m) / ln 2
    facc = fmaf(cv, fmaf(-x, d, fmaxf(d, 0.f) + __builtin_amdgcn_logf(1.f + e)), facc);
    return (d >= 0.f ? inv : e * inv) - x;
  }
  __device__ __forceinline__ static float fr(float x, float d, float& facc) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(d));
    const float inv = __builtin_amdgcn_rcpf(1.f + e);
    facc = fmaf(-x, d, facc + (fmaxf(d, 0.f) + __builtin_amdgcn_logf(1.f + e)));
    return (d >= 0.f ? inv : e * inv) - x;
  }
};

template <>
struct MLoss<kGaussianId> : MLoss<kGaussian> {};

// Identity- and odds-link losses (m >= 0): the model is used as it is.
template <>
struct MLoss<kPoissonId> {
  static constexpr float kM = 1.f, kY = 1.f, kF = 1.f;
  __device__ __forceinline__ static float y(float x, float d) {
    return 1.f - x * __builtin_amdgcn_rcpf(d + (float)kLossEps);
  }
  __device__ __forceinline__ static float fy(float x, float d, float cv, float& facc) {
    const float me = d + (float)kLossEps;
    facc = fmaf(cv, fmaf(-x, __logf(me), d), facc);   // m - x log(m + eps)
    return 1.f - x * __builtin_amdgcn_rcpf(me);
  }
  __device__ __forceinline__ static float fr(float x, float d, float& facc) {
    const float me = d + (float)kLossEps;
    facc = fmaf(-x, __logf(me), facc + d);
    return 1.f - x * __builtin_amdgcn_rcpf(me);
  }
};

template <>
struct MLoss<kBernoulliOdds> {
  static constexpr float kM = 1.f, kY = 1.f, kF = 1.f;
  __device__ __forceinline__ static float y(float x, float d) {
    return __builtin_amdgcn_rcpf(d + 1.f) - x * __builtin_amdgcn_rcpf(d + (float)kLossEps);
  }
  __device__ __forceinline__ static float fy(float x, float d, float cv, float& facc) {
    const float me = d + (float)kLossEps;
    facc = fmaf(cv, fmaf(-x, __logf(me), __logf(d + 1.f)), facc);   // log(m + 1) - x log(m + eps)
    return __builtin_amdgcn_rcpf(d + 1.f) - x * __builtin_amdgcn_rcpf(me);
  }
  __device__ __forceinline__ static float fr(float x, float d, float& facc) {
    const float me = d + (float)kLossEps;
    facc = fmaf(-x, __logf(me), facc + __logf(d + 1.f));
    return __builtin_amdgcn_rcpf(d + 1.f) - x * __builtin_amdgcn_rcpf(me);
  }
};

// One workgroup's tile: pair blocks wgi*8 .. wgi*8+7 of the stream, output
// slot wgi.  sm: LDS scratch of lds_floats(RT, NH, WV) floats; cl: c_h table in LDS.
// Registers / GEMM2 K-steps of the last h-tile that hold slices of the window
// (NK = 0: decided at run time from ns; 1..4: fixed by the instantiation, so
// the skipped work leaves no branches in the pair loop).
template <int NK, int NH>
__device__ __forceinline__ bool reg_active(int ht, int r, int ns) {
  if constexpr (NK == 0)
    return 16 * ht + 4 * r < ns;
  else
    return ht < NH - 1 || r < NK;
}

// XB: the slices are bit-packed binary data (rows of rpw 32-bit words,
// entry i3 is bit i3 % 32 of word i3 / 32, X_t and the window alike).  A
// stage then holds one word per slice row (the row's 32-entry group) and
// the values are unpacked when the stage is read.
// PK = 2: a window of at most 8 slices, two pairs per step.  GEMM1's 16
// rows hold slot 8p + h for slice h of the step's pair p (accumulator
// registers 0-1: pair A, 2-3: pair B), so the model, the loss terms and
// GEMM2's K-steps carry no padding rows; GEMM2 splits its K-steps by pair
// (0-1: A, 2-3: B), and the mode products follow per pair.
template <int LOSS, int RT, int NH, int DMA16, int NK = 0, bool XB = false, int PK = 1, int WV = kWaves>
__device__ __forceinline__ void mfma_tile(const TileArgs& a, const int wgi, float* g1s, float* g2s, float* sm,
                                          float* ring, const float* cl, float* a3t, const int chunk = 0) {
  static_assert(!XB || (NH <= 2 && DMA16 == 0), "bit-packed slices take the staged 4-byte path");
  static_assert(PK == 1 || (PK == 2 && NH == 1), "two pairs per step: one h-tile");
  // DMA16: copy mode of the staged slice rows (0: 4-byte copies; 1: 16-byte
  // copies of the stored rows, the current slice's rows by 4-byte copies of
  // their own (XS); 2: 16-byte copies of every row)
  constexpr bool XS = DMA16 == 1 && !XB;
  constexpr int NT = RT / 4;   // K steps of GEMM1 = j slots per lane
  constexpr int NM = RT / 16;  // M tiles of GEMM2
  constexpr int LOGNT = NT == 4 ? 2 : 3;
  constexpr int NU = 2;                 // 16-entry tiles per group (register budget)
  constexpr int SW = 16 * NU;           // entries per full group

  // G1/G2 rows of each wave's block and the staging ring are LDS arrays of
  // their own (declared by the kernel): reads of the row accumulators then
  // cannot alias the in-flight direct-to-LDS copies, so the compiler adds no
  // wait for those copies inside the pair loop
  float(*g1w)[kTB][RT] = reinterpret_cast<float(*)[kTB][RT]>(g1s);
  float(*g2w)[kTB][RT] = reinterpret_cast<float(*)[kTB][RT]>(g2s);
  float(*g3x)[RT + 1] = reinterpret_cast<float(*)[RT + 1]>(sm);  // SW rows used
  float(*gsx)[RT] = reinterpret_cast<float(*)[RT]>(sm + lds_gs_offset(RT, NH));
  constexpr int NTH = 64 * WV;
  float* lsx = sm + lds_gs_offset(RT, NH) + WV * RT;

  const int tid = threadIdx.x;
  // the wave index is uniform across the wave: keeping it scalar keeps all
  // tile bookkeeping below in scalar registers and branches uniform
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 15, g = lane >> 4;
  // this wave's staging ring (NH <= 2)
  float* ring_w = ring + wave * kStages * stage_floats(NH, PK, RT);
  const int R = a.R, ns = a.ns, I1 = a.I1, I2 = a.I2, I3 = a.I3;
  const int blk = wgi * WV + wave;
  const bool active = blk < a.nblocks;
  const int b1 = active ? blk / a.nb2 : 0, b2 = active ? blk % a.nb2 : 0;
  const int i10 = b1 * a.tb1, i20 = b2 * a.tb2;
  const int n1 = active ? min(a.tb1, I1 - i10) : 0;
  const int n2 = active ? min(a.tb2, I2 - i20) : 0;
  const bool want_loss = a.want & kWantLoss;

  // j held by this lane at GEMM1 step t; clamped index and 0/1 mask make the
  // factor-row loads branch-free when R is not a multiple of the rank tile
  int jt[NT], jc[NT];
  float jm[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    jt[t] = 16 * (t >> 2) + 4 * g + (t & 3);
    jc[t] = min(jt[t], R - 1);
    jm[t] = jt[t] < R ? 1.f : 0.f;
  }
  // column j = 16 mt + n of GEMM2's transposed output held by this lane
  int jn[NM], jnc[NM];
  float jnm[NM];
#pragma unroll
  for (int mt = 0; mt < NM; ++mt) {
    jn[mt] = 16 * mt + n;
    jnc[mt] = min(jn[mt], R - 1);
    jnm[mt] = jn[mt] < R ? 1.f : 0.f;
  }

  // weights as MFMA operands (zero outside h < ns, j < R)
  auto sval = [&](int h, int j) -> float {
    return (h < ns && j < R) ? (h == 0 ? a.st[j] : a.shist[(size_t)(h - 1) * R + j]) : 0.f;
  };
  // Slice order inside an h-tile: row i of GEMM1's A operand holds slice
  // 16 ht + 4 (i % 4) + i / 4, so accumulator register r of lane group g
  // holds slice 16 ht + 4 r + g.  Each register (and each K-step of GEMM2)
  // then covers four consecutive slices, and registers / K-steps lying
  // wholly past the window are skipped with uniform branches.
  float A1op[NH][NT], A2op[NM][NH][4], cv[NH][4];
  // base pointer of the slice each (h-tile, register) row of this lane reads
  const float* sb[NH][4];
  bool hv[NH][4], sr[NH][4];   // row inside the window; row is a stored slice
  // slice held by a row slot (PK = 2: slot 8p + h, slice h of pair p)
  auto slot_slice = [](int slot) { return PK == 2 ? (slot & 7) : slot; };
#pragma unroll
  for (int ht = 0; ht < NH; ++ht) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      A1op[ht][t] = MLoss<LOSS>::kM * sval(slot_slice(16 * ht + 4 * (n & 3) + (n >> 2)), jt[t]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int h = slot_slice(16 * ht + 4 * r + g);
      cv[ht][r] = h < ns ? cl[h] : 0.f;
      hv[ht][r] = h < ns;
      sb[ht][r] = (h == 0 || h >= ns) ? a.Xt : a.ring + (size_t)(h - 1) * a.rstride;
      sr[ht][r] = h >= 1 && h < ns;
    }
    // GEMM2's A operand carries the history weight: c_h S[h][j]
#pragma unroll
    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int h = slot_slice(16 * ht + 4 * t + g);
        A2op[mt][ht][t] = MLoss<LOSS>::kY * (h < ns ? cl[h] : 0.f) * sval(h, 16 * mt + n);
      }
  }

  for (int idx = lane; idx < kTB * RT; idx += 64) {
    (&g1w[wave][0][0])[idx] = 0.f;
    (&g2w[wave][0][0])[idx] = 0.f;
  }
  if constexpr (NH <= 2) {
    // slice rows past the window are never loaded into the ring; they must
    // hold finite values (their products are multiplied by zero weights)
    for (int idx = lane; idx < kStages * stage_floats(NH, PK, RT); idx += 64) ring_w[idx] = 0.f;
    // the zeros must land before any direct-to-LDS copy into the ring
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#endif
  }
  // Staged loads (NH <= 2).  With 16-byte copies (copy mode 1 or 2)
  // instruction k covers LDS rows 8k .. 8k+7, lane l copying 4 values of row
  // 8k + l/8; with 4-byte copies instruction k covers rows 2k, 2k+1, lane l
  // copying value l%32 of row 2k + l/32.  Slice h >= 1 lies at ring + (h-1)
  // omega, slice 0 is the current slice (its LDS row in copy mode 1: see the
  // stage layout above).
  const int hsub = DMA16 != 0 ? (lane >> 3) : (lane >> 5);   // row within an instruction
  const int esub = DMA16 != 0 ? 4 * (lane & 7) : (lane & 31); // entry within the 32-entry group
  float gsacc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) gsacc[t] = 0.f;
  Kahan<float> lacc;

  const int nfull = I3 / SW;
  const int tail = I3 - SW * nfull;
  const int nsc = nfull + (tail > 0 ? 1 : 0);
  const bool vec = (I3 % NU) == 0;
  const int npairs = n1 * n2;

  // groups of this workgroup's I3 chunk
  const int sc_end = min(nsc, (chunk + 1) * a.gpc);
  for (int sc = chunk * a.gpc; sc < sc_end; ++sc) {
    const bool wide = sc < nfull;
    const int c0 = SW * sc;
    const int nu = wide ? NU : (tail + 15) >> 4;
    // entries held by this lane: NU adjacent ones in a full group (and in
    // every group of the staged path but a tail of at most 16 entries), else
    // one per 16-entry tile.  A staged tail of at most 16 entries is
    // computed with one tile only (HALF below).
    const bool half = NH <= 2 && !wide && tail <= 16;
    const bool adj = (wide || NH <= 2) && !half;
    int i3u[NU];
    bool vu[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      i3u[u] = c0 + (adj ? NU * n + u : 16 * u + n);
      vu[u] = (adj || u < nu) && i3u[u] < I3;
    }
    // A3 rows of the group in GEMM1's operand layout (entry of column n,
    // j = jt[t]) and in GEMM2's transposed output layout (entry of column
    // 4g + r, j = 16 mt + n); G3 accumulates in the second layout
    float g3T[NU][NM][4];
    // entry (offset from c0) of output row 4g + r of tile u
    auto eT = [&](int u, int r) { return adj ? NU * (4 * g + r) + u : 16 * u + 4 * g + r; };
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) g3T[u][mt][r] = 0.f;
    // The group's A3 values (zero outside the row and past R) in both
    // layouts, written by the whole workgroup: every wave is at this group,
    // and the previous group's last reads of the arrays came before the
    // barrier that ended it.  Entry of column c of tile u: c0 + NU c + u
    // (adjacent entries per lane) or c0 + 16 u + c.
    float* a3g = a3t + 2 * RT * kA3TPitch;
    for (int idx = tid; idx < NU * RT * 16; idx += NTH) {
      const int u = idx / (RT * 16), j = (idx / 16) % RT, col = idx % 16;
      const int e = adj ? NU * col + u : 16 * u + col;
      const bool ok = (adj || u < nu) && c0 + e < I3 && j < R;
      const float v = ok ? a.A3[(size_t)(c0 + e) * R + j] : 0.f;
      a3t[(u * RT + j) * kA3TPitch + col] = v;
      a3g[(u * 16 + col) * a3g_pitch(RT) + j] = v;
    }
    __syncthreads();
    // GEMM1's operand values of this lane: column n of tile u, j = jt[t]
    auto a3row = [&](int u, float (&out)[NT]) {
#pragma unroll
      for (int t4 = 0; t4 < NT / 4; ++t4) {
        const f4 v = *reinterpret_cast<const f4*>(a3g + (u * 16 + n) * a3g_pitch(RT) + 16 * t4 + 4 * g);
#pragma unroll
        for (int r = 0; r < 4; ++r) out[4 * t4 + r] = v[r];
      }
    };
    // every entry of the group is inside the row (no tail lanes to mask)
    const bool allv = wide && adj;
    float floss = 0.f;

    // Software pipeline over the block's pairs: the loads of pair q+1 (slice
    // values and factor rows) are issued before pair q is computed.  Loads
    // are unconditional or masked-after-zeroing so that no control-flow join
    // forces an early wait on them, and the compute part issues none.
    // VEC: a full group of rows whose start is NU-aligned (one NU-wide load
    // per lane and slice); otherwise per-entry loads.
    auto run_pairs = [&](auto vec_tag, auto half_tag) {
      constexpr bool VEC = decltype(vec_tag)::value;
      constexpr bool HALF = decltype(half_tag)::value;   // one 16-entry tile (staged tail)
      constexpr int NUA = HALF ? 1 : NU;                  // tiles computed
      // Prefetch buffers hold raw loaded values only: any arithmetic on them
      // at load time would force a wait for the loads.
      struct Buf {
        float x[NH][4][NU], a1[NT], a2[NT], a1n[NM], a2n[NM];
        float b1[PK == 2 ? NT : 1], b2[PK == 2 ? NT : 1], b1n[NM], b2n[NM];   // PK = 2: pair B's rows
      };
      Buf bA, bB;
      auto load_pair = [&](int q, Buf& b) {
        const int i1 = i10 + q / n2, i2 = i20 + (q - (q / n2) * n2);
        const float* r1 = a.A1 + (size_t)i1 * R;
        const float* r2 = a.A2 + (size_t)i2 * R;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          b.a1[t] = r1[jc[t]];
          b.a2[t] = r2[jc[t]];
        }
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          b.a1n[mt] = r1[jnc[mt]];
          b.a2n[mt] = r2[jnc[mt]];
        }
        const size_t base_x = ((size_t)i1 * I2 + i2) * I3, base_r = ((size_t)i1 * I2 + i2) * a.rp3;
#pragma unroll
        for (int ht = 0; ht < NH; ++ht)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t base = sr[ht][r] ? base_r : base_x;
            if constexpr (VEC) {
              f2 v = {0.f, 0.f};
              if (hv[ht][r])
                v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(sb[ht][r] + base + c0 + 2 * n));
              b.x[ht][r][0] = v[0];
              b.x[ht][r][1] = v[1];
            } else {
#pragma unroll
              for (int u = 0; u < NU; ++u) {
                float v = 0.f;
                if (hv[ht][r] && vu[u]) v = sb[ht][r][base + i3u[u]];
                b.x[ht][r][u] = v;
              }
            }
          }
      };

      auto compute = [&](int i1l, int i2l, const Buf& b) {
        float W[NT];
#pragma unroll
        // staged factor rows are zero past R; the register-prefetch path
        // reads clamped columns and masks them here
        for (int t = 0; t < NT; ++t) W[t] = NH <= 2 ? b.a1[t] * b.a2[t] : b.a1[t] * b.a2[t] * jm[t];
        float a1n[NM], a2n[NM], Wn[NM];
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          a1n[mt] = NH <= 2 ? b.a1n[mt] : b.a1n[mt] * jnm[mt];
          a2n[mt] = NH <= 2 ? b.a2n[mt] : b.a2n[mt] * jnm[mt];
          Wn[mt] = a1n[mt] * a2n[mt];
        }

        // GEMM1: model values for 16 h x 16 entries per (h-tile, entry tile).
        // The pair's weights W multiply whichever operand has fewer values
        // per lane (the weight rows with one h-tile, else the entries).
        constexpr bool kWA = NH < NU;
        float Aw[kWA ? NH : 1][NT];
        if constexpr (kWA) {
#pragma unroll
          for (int ht = 0; ht < NH; ++ht)
#pragma unroll
            for (int t = 0; t < NT; ++t) Aw[ht][t] = A1op[ht][t] * W[t];
        }
        float a3r[NU][NT];
#pragma unroll
        for (int u = 0; u < NUA; ++u) a3row(u, a3r[u]);
        f4 D1[NH][NU];
#pragma unroll
        for (int ht = 0; ht < NH; ++ht)
#pragma unroll
          for (int u = 0; u < NUA; ++u) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            // the Gaussian identity path takes m = 0 here (y = -2x)
            if (LOSS != kGaussianId && (VEC || u < nu)) {
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if constexpr (kWA)
                  acc = mfma(Aw[ht][t], a3r[u][t], acc);
                else
                  acc = mfma(A1op[ht][t], W[t] * a3r[u][t], acc);
              }
            }
            D1[ht][u] = acc;
          }

        // loss derivative in place, and the objective terms of the group
        // weighted by c_h, summed per entry tile and added to the lane's
        // running sum with compensation.  Padded slices (c_h = 0) have zero
        // weight rows, so d = 0 and a finite x give finite terms that the
        // zero weight removes.  Entries past the end of a row (tail lanes)
        // need no mask in y: their A3 values are zero, so every product that
        // uses them vanishes and their mode-3 rows are never written; their
        // objective terms are dropped per entry tile.
        // Registers holding only slices past the window are left as they
        // are: GEMM2 skips their K-steps.
        if (want_loss) {
          // weighted terms summed in one register over the pairs of a row
          // of the block; the row's sum joins the compensated lane total
          if (allv) {
#pragma unroll
            for (int ht = 0; ht < NH; ++ht)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (!reg_active<NK, NH>(ht, r, ns)) continue;
#pragma unroll
                for (int u = 0; u < NUA; ++u)
                  D1[ht][u][r] = MLoss<LOSS>::fy(b.x[ht][r][u], D1[ht][u][r], cv[ht][r], floss);
              }
          } else {
#pragma unroll
            for (int ht = 0; ht < NH; ++ht)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (!reg_active<NK, NH>(ht, r, ns)) continue;
#pragma unroll
                for (int u = 0; u < NUA; ++u) {
                  float f = 0.f;
                  D1[ht][u][r] = MLoss<LOSS>::fy(b.x[ht][r][u], D1[ht][u][r], cv[ht][r], f);
                  floss += vu[u] ? f : 0.f;
                }
              }
          }
          if (i2l == n2 - 1) {
            lacc.add(floss);
            floss = 0.f;
          }
        } else {
#pragma unroll
          for (int ht = 0; ht < NH; ++ht)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (!reg_active<NK, NH>(ht, r, ns)) continue;
#pragma unroll
              for (int u = 0; u < NUA; ++u) D1[ht][u][r] = MLoss<LOSS>::y(b.x[ht][r][u], D1[ht][u][r]);
            }
        }

        // temporal-weight gradient: y_t sits in register 0 of lane group 0
        {
          float ps[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) ps[t] = 0.f;
#pragma unroll
          for (int u = 0; u < NUA; ++u) {
            const float yt = __shfl(D1[0][u][0], n);
#pragma unroll
            for (int t = 0; t < NT; ++t) ps[t] += yt * a3r[u][t];
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) gsacc[t] += W[t] * ps[t];
        }

        // GEMM2, transposed: yhat[e][j] = sum_h y[h][e] (c_h S[h][j]).  GEMM1's
        // accumulator is the A operand (rows e, K = h) and the weights are
        // the B operand, so register r of lane (g, n) holds entry row 4g + r
        // and column j = 16 mt + n: the sum over the entries for V is four
        // in-lane terms and two lane-swap steps.
        float Vp[NM];
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) Vp[mt] = 0.f;
#pragma unroll
        for (int u = 0; u < NUA; ++u) {
          if (!VEC && u >= nu) continue;
#pragma unroll
          for (int mt = 0; mt < NM; ++mt) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ht = 0; ht < NH; ++ht)
#pragma unroll
              for (int t = 0; t < 4; ++t)
                if (reg_active<NK, NH>(ht, t, ns)) acc = mfma(D1[ht][u][t], A2op[mt][ht][t], acc);
            const f4 a3v = *reinterpret_cast<const f4*>(a3t + (u * RT + jn[mt]) * kA3TPitch + 4 * g);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              g3T[u][mt][r] += acc[r] * Wn[mt];
              Vp[mt] += acc[r] * a3v[r];
            }
          }
        }
        // the rows belong to this wave alone and its LDS adds complete in
        // program order, so the sums are deterministic; the adds return
        // nothing, so the wave does not wait for them
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          const float v = sum_lane_groups(Vp[mt]);
          if (g == 0 && jn[mt] < R) {
            lds_add(&g1w[wave][i1l][jn[mt]], v * a2n[mt]);
            lds_add(&g2w[wave][i2l][jn[mt]], v * a1n[mt]);
          }
        }
      };

      // PK = 2: pairs A (local i1 ai1, i2 ai2) and B (bi1, bi2; bvalid false
      // past the block's last pair, whose rows are then pair A's again) in
      // one 16-row tile: slot 8p + h holds slice h of pair p.
      auto compute2 = [&](int ai1, int ai2, int bi1, int bi2, bool bvalid, const Buf& b) {
        float WA[NT], WB[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          WA[t] = b.a1[t] * b.a2[t];
          WB[t] = bvalid ? b.b1[t] * b.b2[t] : 0.f;
        }
        float WnA[NM], WnB[NM];
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          WnA[mt] = b.a1n[mt] * b.a2n[mt];
          WnB[mt] = b.b1n[mt] * b.b2n[mt];
        }
        // GEMM1's A operand: row n holds slot 4 (n % 4) + n / 4, pair B for
        // n % 4 >= 2
        const bool rowb = (n & 2) != 0;
        float Aw[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) Aw[t] = A1op[0][t] * (rowb ? WB[t] : WA[t]);
        float a3r[NU][NT];
#pragma unroll
        for (int u = 0; u < NUA; ++u) a3row(u, a3r[u]);
        f4 D1[NU];
#pragma unroll
        for (int u = 0; u < NUA; ++u) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
          if (LOSS != kGaussianId) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc = mfma(Aw[t], a3r[u][t], acc);
          }
          D1[u] = acc;
        }
        // register r holds slice 4 (r % 2) + g of pair r / 2; registers 1
        // and 3 hold slices 4..7, used only when the window has more than 4
        const bool hi = ns > 4;
        if (want_loss) {
          float fl = 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if ((r & 1) && !hi) continue;
#pragma unroll
            for (int u = 0; u < NUA; ++u) {
              float f = 0.f;
              D1[u][r] = MLoss<LOSS>::fy(b.x[0][r][u], D1[u][r], cv[0][r], f);
              fl += (vu[u] && (r < 2 || bvalid)) ? f : 0.f;
            }
          }
          lacc.add(fl);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if ((r & 1) && !hi) continue;
#pragma unroll
            for (int u = 0; u < NUA; ++u) D1[u][r] = MLoss<LOSS>::y(b.x[0][r][u], D1[u][r]);
          }
        }
        // temporal-weight gradient: y_t of pair A in register 0, of pair B
        // in register 2 (lane group 0)
        {
          float psA[NT], psB[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) psA[t] = psB[t] = 0.f;
#pragma unroll
          for (int u = 0; u < NUA; ++u) {
            const float ya = __shfl(D1[u][0], n), yb = __shfl(D1[u][2], n);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              psA[t] += ya * a3r[u][t];
              psB[t] += yb * a3r[u][t];
            }
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) gsacc[t] += WA[t] * psA[t] + WB[t] * psB[t];
        }
        // GEMM2, transposed, per pair: K-steps 0-1 are pair A's slices,
        // 2-3 pair B's
        float VpA[NM], VpB[NM];
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) VpA[mt] = VpB[mt] = 0.f;
#pragma unroll
        for (int u = 0; u < NUA; ++u) {
#pragma unroll
          for (int mt = 0; mt < NM; ++mt) {
            f4 accA = {0.f, 0.f, 0.f, 0.f}, accB = {0.f, 0.f, 0.f, 0.f};
            accA = mfma(D1[u][0], A2op[mt][0][0], accA);
            accB = mfma(D1[u][2], A2op[mt][0][2], accB);
            if (hi) {
              accA = mfma(D1[u][1], A2op[mt][0][1], accA);
              accB = mfma(D1[u][3], A2op[mt][0][3], accB);
            }
            const f4 a3v = *reinterpret_cast<const f4*>(a3t + (u * RT + jn[mt]) * kA3TPitch + 4 * g);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              g3T[u][mt][r] += accA[r] * WnA[mt] + (bvalid ? accB[r] * WnB[mt] : 0.f);
              VpA[mt] += accA[r] * a3v[r];
              VpB[mt] += accB[r] * a3v[r];
            }
          }
        }
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          const float va = sum_lane_groups(VpA[mt]);
          const float vb = sum_lane_groups(VpB[mt]);
          if (g == 0 && jn[mt] < R) {
            lds_add(&g1w[wave][ai1][jn[mt]], va * b.a2n[mt]);
            lds_add(&g2w[wave][ai2][jn[mt]], va * b.a1n[mt]);
            if (bvalid) {
              lds_add(&g1w[wave][bi1][jn[mt]], vb * b.b2n[mt]);
              lds_add(&g2w[wave][bi2][jn[mt]], vb * b.b1n[mt]);
            }
          }
        }
      };

      if constexpr (VEC && NH <= 2) {
        // Staged pipeline: the slice rows and factor rows of pair q are
        // copied global -> LDS by the direct-to-LDS loads two pairs ahead;
        // these are the only vector-memory operations of the loop, so the
        // wave waits for exactly the stage it is about to read.  Every stage
        // takes the same KX + 1 copy instructions (rows past the window copy
        // a valid row into padding that is never used), so the waits are
        // compile-time constants.
        constexpr int KX = XB ? 1 : (DMA16 != 0 ? 2 * NH : 8 * NH);   // slice-row copies per stage
        // + the factor rows (one copy, or one per pair at rank tile 32),
        // + the current slice's rows (XS: one copy per pair)
        constexpr int K = KX + (PK == 2 && RT > 16 ? 2 : 1) + (XS ? PK : 0);
        constexpr int SFP = stage_floats(NH, PK, RT);
        // entries past the end of the row copy from the group start instead
        // (finite values whose terms are masked)
        const size_t eoff = (size_t)(c0 + esub < I3 ? c0 + esub : c0);
        // XS: entry of the current slice's row copied by this lane
        const size_t xoff = (size_t)(c0 + (lane & 31) < I3 ? c0 + (lane & 31) : c0);
        // 16-byte copies of stored slice s (window slot s - 1) at LDS row
        // s - 1: the lane's address is base + pair x pitch (bytes), a single
        // 32 x 32 -> 64-bit multiply-add per copy (pair < 2^32).  Rows past
        // the window copy a row of zeros (pitch 0) that no term uses; the
        // lanes of a pair's last row copy nothing (the current slice's row
        // goes there).  Stored rows keep I3 rounded up to 32 values, so a
        // 16-byte piece never leaves its row; the values past I3 are zero.
        uint64_t src16[DMA16 != 0 ? KX : 1];
        uint32_t pit16[DMA16 != 0 ? KX : 1];
        if constexpr (XS) {
#pragma unroll
          for (int k = 0; k < KX; ++k) {
            // PK = 2: copy k carries stored slice hsub + 1 of pair k
            const int h = (PK == 2 ? hsub : 8 * k + hsub) + 1;
            const bool stored = h < ns;
            src16[k] = stored ? reinterpret_cast<uint64_t>(a.ring + (size_t)(h - 1) * a.rstride + eoff)
                              : reinterpret_cast<uint64_t>(g_zero_row + esub);
            pit16[k] = stored ? 4u * (uint32_t)a.rp3 : 0u;
          }
        } else if constexpr (DMA16 == 2) {
          // every row 16-byte aligned (I3 a multiple of 4): slice h at row h,
          // rows past the window copy the current slice's row again
#pragma unroll
          for (int k = 0; k < KX; ++k) {
            // PK = 2: copy k carries slice hsub of pair k
            const int h = PK == 2 ? hsub : 8 * k + hsub;
            const bool stored = h >= 1 && h < ns;
            src16[k] = reinterpret_cast<uint64_t>(stored ? a.ring + (size_t)(h - 1) * a.rstride + eoff : a.Xt + eoff);
            pit16[k] = 4u * (stored ? (uint32_t)a.rp3 : (uint32_t)I3);
          }
        }
        // 4-byte copies: rows 2k + hsub; base pointers for hsub = 0 / 1 of
        // the ring part, the k-dependent offset is scalar
        const float* ringl = a.ring + (size_t)hsub * a.rstride + eoff;   // row 2k+hsub = ringl + (2k-1) rstride
        const float* xtl = a.Xt + eoff;
        // pair of copy step p (row-major over the block), advanced incrementally
        int pi1 = 0, pi2 = 0;
        // bit-packed rows: lane l copies the group's word of row slot l, slice
        // l (PK = 2: slice l % 8 of pair l / 8); rows past the window copy
        // the current slice's word
        const int wsl = PK == 2 ? (lane & 7) : lane;
        const uint32_t* wrow = reinterpret_cast<const uint32_t*>(
                                   (wsl == 0 || wsl >= ns || (PK == 2 && lane >= 16))
                                       ? a.Xt
                                       : a.ring + (size_t)(wsl - 1) * a.rstride) +
                               c0 / 32;
        // stage st's pairs: (pi1, pi2) and, with PK = 2, the next pair of the
        // block (the same pair again past the block's last pair: its values
        // are loaded but never used)
        auto issue = [&](int st) {
          const int a1i = i10 + pi1, a2i = i20 + pi2;
          if (++pi2 == n2) {
            pi2 = 0;
            ++pi1;
          }
          int b1i = a1i, b2i = a2i;
          if constexpr (PK == 2) {
            if (pi1 < n1) {
              b1i = i10 + pi1;
              b2i = i20 + pi2;
              if (++pi2 == n2) {
                pi2 = 0;
                ++pi1;
              }
            }
          }
          const size_t pair = (size_t)a1i * I2 + a2i, pairb = (size_t)b1i * I2 + b2i;
          float* stg = ring_w + st * SFP;
          if constexpr (XB) {
            const size_t pw = PK == 2 && (lane & 8) ? pairb : pair;
            load_to_lds(reinterpret_cast<const float*>(wrow + pw * (size_t)a.rpw), stg, 4);
          } else if constexpr (DMA16 != 0) {
#pragma unroll
            for (int k = 0; k < KX; ++k) {
              const uint32_t p32 = (uint32_t)(PK == 2 && k == 1 ? pairb : pair);
              const float* src = reinterpret_cast<const float*>((uint64_t)p32 * pit16[k] + src16[k]);
              if constexpr (XS) {
                // lanes 56-63 of the copy holding a pair's last row
                if ((PK == 2 || k == KX - 1) && lane >= 56) continue;
              }
              load_to_lds(src, stg + 256 * k, 16);
            }
            if constexpr (XS) {
              // the current slice's rows, 32 lanes per pair
              if (lane < 32) {
                load_to_lds(a.Xt + pair * (size_t)I3 + xoff, stg + (PK == 2 ? 7 : 16 * NH - 1) * 32, 4);
                if constexpr (PK == 2) load_to_lds(a.Xt + pairb * (size_t)I3 + xoff, stg + 15 * 32, 4);
              }
            }
          } else {
#pragma unroll
            for (int k = 0; k < KX; ++k) {
              // PK = 2: copies 0-3 carry pair A's slices 2k + hsub, 4-7 pair B's
              const int kk = PK == 2 ? (k & 3) : k;
              const size_t pk = PK == 2 && k >= 4 ? pairb : pair;
              const int h = 2 * kk + hsub;
              const bool stored = h >= 1 && h < ns;
              const float* sp = stored ? ringl + ((size_t)(2 * kk - 1) * a.rstride + pk * a.rp3) : xtl + pk * I3;
              load_to_lds(sp, stg + 64 * k, 4);
            }
          }
          // factor rows: lanes 0-31 copy row i1 of A1, lanes 32-63 row i2 of
          // A2; columns j >= R are never written and keep their zeros.  Two
          // pairs at rank tile 16: lanes 16-31 / 48-63 copy pair B's rows
          // into the upper halves; at rank tile 32 a second copy follows.
          if constexpr (PK == 2 && RT <= 16) {
            const int col = lane & 15;
            const bool pb = (lane & 16) != 0;
            if (col < R) {
              const float* fsrc = lane < 32 ? a.A1 + (size_t)(pb ? b1i : a1i) * R + col
                                            : a.A2 + (size_t)(pb ? b2i : a2i) * R + col;
              load_to_lds(fsrc, stg + 512 * NH, 4);
            }
          } else if ((lane & 31) < R) {
            const float* fsrc = lane < 32 ? a.A1 + (size_t)a1i * R + lane : a.A2 + (size_t)a2i * R + (lane - 32);
            load_to_lds(fsrc, stg + 512 * NH, 4);
            if constexpr (PK == 2) {
              const float* fsrcb = lane < 32 ? a.A1 + (size_t)b1i * R + lane : a.A2 + (size_t)b2i * R + (lane - 32);
              load_to_lds(fsrcb, stg + 512 * NH + pair_b_offset(RT), 4);
            }
          }
        };
        // steps of the loop: one pair each, or two with PK = 2
        const int nsteps = PK == 2 ? (npairs + 1) / 2 : npairs;
        if (nsteps > 0) issue(0);
        if (nsteps > 1) issue(1);
        int ci1 = 0, ci2 = 0;
        // step q uses stage q % kStages; the loop is unrolled by kStages so
        // that every stage offset is a constant of the LDS instructions
        auto step = [&](auto stage_tag, int q) {
          constexpr int st = decltype(stage_tag)::value;
          if (q + 2 < nsteps) {
            issue((st + 2) % kStages);
            wait_vmcnt(2 * K);
          } else if (q + 1 < nsteps) {
            wait_vmcnt(K);
          } else {
            wait_vmcnt(0);
          }
          const float* stg = ring_w + st * SFP;
          // LDS offset of the row read by register r of h-tile ht: slice
          // row 16 ht + 4 r + g, or with XS stored slice s at row s - 1 and
          // the current slice in the pair's last row
          auto xrow = [&](int ht, int r) -> int {
            if constexpr (!XS) {
              return (16 * ht + 4 * r + g) * 32;
            } else if constexpr (PK == 2) {
              const int p = r >> 1, h = 4 * (r & 1) + g;
              return (h == 0 ? 8 * p + 7 : 8 * p + h - 1) * 32;
            } else {
              const int slot = 16 * ht + 4 * r + g;
              return (slot == 0 ? 16 * NH - 1 : slot - 1) * 32;
            }
          };
          Buf b;
#pragma unroll
          for (int ht = 0; ht < NH; ++ht)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if constexpr (XB) {
                // entries c0 + n (one tile) or c0 + 2n + u of the row's word
                const uint32_t w = reinterpret_cast<const uint32_t*>(stg)[16 * ht + 4 * r + g];
                if constexpr (HALF) {
                  b.x[ht][r][0] = (float)((w >> n) & 1u);
                  b.x[ht][r][1] = 0.f;
                } else {
                  b.x[ht][r][0] = (float)((w >> (2 * n)) & 1u);
                  b.x[ht][r][1] = (float)((w >> (2 * n + 1)) & 1u);
                }
              } else if constexpr (HALF) {
                b.x[ht][r][0] = stg[xrow(ht, r) + n];
                b.x[ht][r][1] = 0.f;
              } else {
                const f2 v = *reinterpret_cast<const f2*>(stg + xrow(ht, r) + 2 * n);
                b.x[ht][r][0] = v[0];
                b.x[ht][r][1] = v[1];
              }
            }
          // columns t of this lane are 16 (t / 4) + 4 g + t % 4: four
          // contiguous values per 16-column tile (zero past R)
          const float* fa = stg + 512 * NH;
#pragma unroll
          for (int t4 = 0; t4 < NT / 4; ++t4) {
            const f4 v1 = *reinterpret_cast<const f4*>(fa + 16 * t4 + 4 * g);
            const f4 v2 = *reinterpret_cast<const f4*>(fa + 32 + 16 * t4 + 4 * g);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              b.a1[4 * t4 + r] = v1[r];
              b.a2[4 * t4 + r] = v2[r];
            }
          }
#pragma unroll
          for (int mt = 0; mt < NM; ++mt) {
            b.a1n[mt] = fa[jn[mt]];
            b.a2n[mt] = fa[32 + jn[mt]];
          }
          if constexpr (PK == 2) {
            const float* fb = fa + pair_b_offset(RT);
#pragma unroll
            for (int t4 = 0; t4 < NT / 4; ++t4) {
              const f4 v1 = *reinterpret_cast<const f4*>(fb + 16 * t4 + 4 * g);
              const f4 v2 = *reinterpret_cast<const f4*>(fb + 32 + 16 * t4 + 4 * g);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                b.b1[4 * t4 + r] = v1[r];
                b.b2[4 * t4 + r] = v2[r];
              }
            }
#pragma unroll
            for (int mt = 0; mt < NM; ++mt) {
              b.b1n[mt] = fb[jn[mt]];
              b.b2n[mt] = fb[32 + jn[mt]];
            }
            // the step's two pairs in the block's row-major order
            const int ai1 = ci1, ai2 = ci2;
            if (++ci2 == n2) {
              ci2 = 0;
              ++ci1;
            }
            const bool bvalid = ci1 < n1;
            compute2(ai1, ai2, ci1, ci2, bvalid, b);
            if (bvalid && ++ci2 == n2) {
              ci2 = 0;
              ++ci1;
            }
          } else {
            compute(ci1, ci2, b);
            if (++ci2 == n2) {
              ci2 = 0;
              ++ci1;
            }
          }
        };
        static_assert(kStages == 3, "the pair loop is unrolled by three");
        for (int q = 0; q < nsteps; q += kStages) {
          step(std::integral_constant<int, 0>{}, q);
          if (q + 1 >= nsteps) break;
          step(std::integral_constant<int, 1>{}, q + 1);
          if (q + 2 >= nsteps) break;
          step(std::integral_constant<int, 2>{}, q + 2);
        }
      } else {
        // ping-pong: the buffer being computed was filled one step earlier
        // while the other buffer's loads are in flight
        if (npairs > 0) load_pair(0, bA);
        for (int q = 0; q < npairs; q += 2) {
          if (q + 1 < npairs) load_pair(q + 1, bB);
          compute(q / n2, q % n2, bA);
          if (q + 1 >= npairs) break;
          if (q + 2 < npairs) load_pair(q + 2, bA);
          compute((q + 1) / n2, (q + 1) % n2, bB);
        }
      }
    };
    using True = std::integral_constant<bool, true>;
    using False = std::integral_constant<bool, false>;
    if constexpr (NH <= 2) {
      if (half)
        run_pairs(True{}, True{});
      else
        run_pairs(True{}, False{});
    } else {
      if (wide && vec)
        run_pairs(True{}, False{});
      else
        run_pairs(False{}, False{});
    }

    if constexpr (NH <= 2) {
      // Every stage of the staging rings is idle here: each wave stores its
      // mode-3 rows of the group in its own ring, and the workgroup adds the
      // waves in order (one barrier round instead of one per wave; the sums
      // are the same, in the same order).
      constexpr int SF = stage_floats(NH, PK, RT);
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int mt = 0; mt < NM; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) ring_w[eT(u, r) * RT + jn[mt]] = g3T[u][mt][r];
      __syncthreads();
      for (int idx = tid; idx < SW * RT; idx += NTH) {
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < WV; ++w) sum += ring[w * kStages * SF + idx];
        const int l = idx / RT, j = idx - (idx / RT) * RT;
        if (c0 + l < I3 && j < R) a.G3p[((size_t)wgi * I3 + c0 + l) * R + j] = sum;
      }
      __syncthreads();
      // the rows may have covered stage 0's factor columns, which must stay
      // zero past R
      if constexpr (SW * RT > 512 * NH) {
        ring_w[512 * NH + lane] = 0.f;
        if constexpr (PK == 2 && RT > 16) ring_w[512 * NH + 64 + lane] = 0.f;
      }
    } else {
      // combine the waves' mode-3 rows of this group in wave order
      for (int idx = tid; idx < SW * (RT + 1); idx += NTH) (&g3x[0][0])[idx] = 0.f;
      __syncthreads();
      for (int w = 0; w < WV; ++w) {
        if (wave == w) {
#pragma unroll
          for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if ((adj || u < nu) && c0 + eT(u, r) < I3)
#pragma unroll
                for (int mt = 0; mt < NM; ++mt) g3x[eT(u, r)][jn[mt]] += g3T[u][mt][r];
        }
        __syncthreads();
      }
      for (int idx = tid; idx < SW * RT; idx += NTH) {
        const int l = idx / RT, j = idx - (idx / RT) * RT;
        if (c0 + l < I3 && j < R) a.G3p[((size_t)wgi * I3 + c0 + l) * R + j] = g3x[l][j];
      }
      __syncthreads();
    }
  }

  // mode-1/2 partial rows of this wave's block
  if (active) {
    for (int idx = lane; idx < kTB * RT; idx += 64) {
      const int l = idx / RT, j = idx - (idx / RT) * RT;
      if (j < R) {
        if (l < n1) a.G1p[(((size_t)chunk * a.nb2 + b2) * I1 + i10 + l) * R + j] = g1w[wave][l][j];
        if (l < n2) a.G2p[(((size_t)chunk * (a.nblocks / a.nb2) + b1) * I2 + i20 + l) * R + j] = g2w[wave][l][j];
      }
    }
  }
  // temporal-weight gradient and objective partials of the workgroup
  {
    float gv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) gv[t] = MLoss<LOSS>::kY * gsacc[t];
    // sum over the 16 lanes of the row, then over the 4 rows
    const float v = row_reduce_scatter<NT>(gv, n);
    float vs = v;
    if ((n & ((16 / NT) - 1)) == 0) {
      const int tt = n >> (4 - LOGNT);
      gsx[wave][16 * (tt >> 2) + 4 * g + (tt & 3)] = vs;
    }
    float ls = MLoss<LOSS>::kF * lacc.s;
    for (int m = 32; m >= 1; m >>= 1) ls += __shfl_xor(ls, m);
    if (lane == 0) lsx[wave] = ls;
  }
  __syncthreads();
  if (tid < R) {
    float s = 0.f;
    for (int w = 0; w < WV; ++w) s += gsx[w][tid];
    a.gsp[((size_t)wgi * a.nch + chunk) * R + tid] = s;
  }
  if (tid == 0) {
    float s = 0.f;
    for (int w = 0; w < WV; ++w) s += lsx[w];
    a.lossp[(size_t)wgi * a.nch + chunk] = s;
  }
}

template <int LOSS, int RT, int NH, int DMA16, int NK, bool XB = false, int PK = 1>
__device__ __forceinline__ void fused_body(const MArgs& a) {
  constexpr int WV = tile_waves(RT);
  __shared__ float g1s[WV * kTB * RT];
  __shared__ float g2s[WV * kTB * RT];
  __shared__ float sm[lds_floats(RT, NH, WV)];
  // the staging ring is an LDS object of its own: the direct-to-LDS copies
  // write only this array
  __shared__ __attribute__((aligned(16))) float ring[ring_floats(NH, PK, RT, WV) > 0 ? ring_floats(NH, PK, RT, WV) : 4];
  __shared__ float cl[kMaxNs];
  __shared__ __attribute__((aligned(16))) float a3t[a3t_floats(RT)];
  for (int h = threadIdx.x; h < kMaxNs; h += 64 * WV) cl[h] = h < a.t.ns ? a.c[h] : 0.f;
  __syncthreads();
  mfma_tile<LOSS, RT, NH, DMA16, NK, XB, PK, WV>(a.t, blockIdx.x / a.t.nch, g1s, g2s, sm, ring, cl, a3t,
                                                 blockIdx.x % a.t.nch);
}

template <int LOSS, int RT, int NH, int DMA16, int NK, bool XB = false, int PK = 1>
__global__ void __launch_bounds__(64 * tile_waves(RT))
__attribute__((amdgpu_waves_per_eu(tile_min_waves<RT, NH, PK, DMA16>(), 8))) fused_dense_mfma(MArgs a) {
  fused_body<LOSS, RT, NH, DMA16, NK, XB, PK>(a);
}

// Rank tile 16 with one h-tile: the LDS of two workgroups fits a compute
// unit, so the register budget is held to 128 (four waves per SIMD); the
// few values that do not fit are spilled outside the pair loop.
template <int LOSS, int DMA16, int NK, bool XB = false, int PK = 1>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
fused_dense_mfma_r16(MArgs a) {
  fused_body<LOSS, 16, 1, DMA16, NK, XB, PK>(a);
}


// One variant's share of the work list: items [begin, end), taken in order
// from the variant's own counter.
template <int LOSS, int RT, int NH, int DMA16, int PK = 1>
__device__ __forceinline__ void batch_grad_body(const BatchDesc* __restrict__ desc,
                                                const BatchState* __restrict__ state,
                                                const int2* __restrict__ items, int begin, int end,
                                                int* __restrict__ counter, int want) {
  __shared__ float g1s[kWaves * kTB * RT];
  __shared__ float g2s[kWaves * kTB * RT];
  __shared__ float sm[lds_floats(RT, NH, kWaves)];
  __shared__ __attribute__((aligned(16))) float ring[ring_floats(NH, PK, RT, kWaves) > 0 ? ring_floats(NH, PK, RT, kWaves) : 4];
  __shared__ float cl[kMaxNs];
  __shared__ __attribute__((aligned(16))) float a3t[a3t_floats(RT)];
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = begin + atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= end) break;
    const int si = items[it].x, wg = items[it].y;
    const BatchDesc& d = desc[si];
    const BatchState& s = state[si];
    TileArgs ta;
    ta.Xt = d.Xt;
    ta.ring = d.ring;
    ta.rstride = (size_t)d.rstride;
    ta.rp3 = (size_t)d.rp3;
    ta.st = d.st;
    ta.shist = d.shist;
    ta.A1 = d.A;
    ta.A2 = d.A + d.fac_off1;
    ta.A3 = d.A + d.fac_off2;
    ta.G1p = d.G1p;
    ta.G2p = d.G2p;
    ta.G3p = d.G3p;
    ta.gsp = d.gsp;
    ta.lossp = d.lossp;
    ta.I1 = d.I1; ta.I2 = d.I2; ta.I3 = d.I3; ta.R = d.R;
    ta.ns = 1 + s.nwin;
    ta.want = want;
    ta.tb1 = d.tb1; ta.tb2 = d.tb2; ta.nb2 = d.nb2; ta.nblocks = d.nblocks;
    ta.nch = 1;
    ta.gpc = 1 << 30;
    for (int h = threadIdx.x; h < kMaxNs; h += kThreads) {
      float v = 0.f;
      if (h == 0) v = 1.f;
      else if (h < ta.ns) v = (float)(d.w * pow(d.theta, (double)(s.t - s.slot_t[h - 1])));
      cl[h] = v;
    }
    __syncthreads();
    // GEMM2 K-steps of the last h-tile fixed per item, as in a single
    // stream's build; a window that has not yet reached the variant's
    // h-tiles keeps the run-time masks
    const int nl = ta.ns - 16 * (NH - 1);
    if (PK != 1 || nl <= 0)
      mfma_tile<LOSS, RT, NH, DMA16, 0, false, PK>(ta, wg, g1s, g2s, sm, ring, cl, a3t);
    else if (nl <= 4)
      mfma_tile<LOSS, RT, NH, DMA16, 1, false, PK>(ta, wg, g1s, g2s, sm, ring, cl, a3t);
    else if (nl <= 8)
      mfma_tile<LOSS, RT, NH, DMA16, 2, false, PK>(ta, wg, g1s, g2s, sm, ring, cl, a3t);
    else if (nl <= 12)
      mfma_tile<LOSS, RT, NH, DMA16, 3, false, PK>(ta, wg, g1s, g2s, sm, ring, cl, a3t);
    else
      mfma_tile<LOSS, RT, NH, DMA16, 4, false, PK>(ta, wg, g1s, g2s, sm, ring, cl, a3t);
    __syncthreads();
  }
}

template <int LOSS, int RT, int NH, int DMA16, int PK = 1>
__global__ void __launch_bounds__(kThreads) batch_grad_kernel(const BatchDesc* __restrict__ desc,
                                                              const BatchState* __restrict__ state,
                                                              const int2* __restrict__ items, int begin, int end,
                                                              int* __restrict__ counter, int want) {
  batch_grad_body<LOSS, RT, NH, DMA16, PK>(desc, state, items, begin, end, counter, want);
}

// Rank tile 16, one h-tile: four waves per SIMD, as fused_dense_mfma_r16.
template <int LOSS, int DMA16, int PK = 1>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
batch_grad_kernel_r16(const BatchDesc* __restrict__ desc, const BatchState* __restrict__ state,
                      const int2* __restrict__ items, int begin, int end, int* __restrict__ counter, int want) {
  batch_grad_body<LOSS, 16, 1, DMA16, PK>(desc, state, items, begin, end, counter, want);
}

template <int LOSS, int RT, int NH>
hipError_t launch(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p, float* gsp,
                  float* lossp) {
  MArgs m;
  TileArgs& a = m.t;
  for (int h = 0; h < kMaxNs; ++h) m.c[h] = h < c.ns ? (float)c.c[h] : 0.f;
  a.Xt = static_cast<const float*>(c.X[0]);
  a.ring = static_cast<const float*>(c.ring);
  a.rstride = c.ring_stride;
  a.rp3 = c.ring_pitch;
  a.st = static_cast<const float*>(c.S[0]);
  a.shist = static_cast<const float*>(c.shist);
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
  a.nch = p.nch;
  a.gpc = p.gpc;
  a.rpw = (c.I3 + 31) / 32;
  // copy mode of the slice rows (16-byte copies need 16-byte aligned rows);
  // nk: registers of the last h-tile that hold slices of the window
  const int cp = copy_mode(c.ring_pitch, c.I3);
  auto by_cp = [&](auto f) {
    switch (cp) {
      case 2: f(std::integral_constant<int, 2>{}); break;
      case 1: f(std::integral_constant<int, 1>{}); break;
      default: f(std::integral_constant<int, 0>{}); break;
    }
  };
  const int nk = (c.ns - 16 * (NH - 1) + 3) / 4;
  constexpr bool kBinary = LOSS == kBernoulliLogit || LOSS == kBernoulliOdds;
  if (c.xbits && (!kBinary || NH > 2)) return hipErrorInvalidValue;
  // a window of at most 8 slices: two pairs per step (PK = 2)
  if constexpr (NH == 1) {
    if (c.xbits && c.ns <= 8) {
      if constexpr (kBinary) {
        if constexpr (RT == 16)
          hipLaunchKernelGGL((fused_dense_mfma_r16<LOSS, 0, 0, true, 2>), dim3(p.nwg * p.nch), dim3(kThreads), 0, c.stream,
                             m);
        else
          hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, 1, 0, 0, true, 2>), dim3(p.nwg * p.nch),
                             dim3(64 * tile_waves(RT)), 0, c.stream, m);
      }
      return hipGetLastError();
    }
    if (c.ns <= 8) {
      by_cp([&](auto cpc) {
        constexpr int CP = decltype(cpc)::value;
        if constexpr (RT == 16)
          hipLaunchKernelGGL((fused_dense_mfma_r16<LOSS, CP, 0, false, 2>), dim3(p.nwg * p.nch), dim3(kThreads), 0, c.stream,
                             m);
        else
          hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, 1, CP, 0, false, 2>), dim3(p.nwg * p.nch),
                             dim3(64 * tile_waves(RT)), 0, c.stream, m);
      });
      return hipGetLastError();
    }
  }
  auto go = [&](auto nkc) {
    constexpr int K = decltype(nkc)::value;
    if constexpr (kBinary && NH <= 2) {
      if (c.xbits) {
        if constexpr (RT == 16 && NH == 1)
          hipLaunchKernelGGL((fused_dense_mfma_r16<LOSS, 0, K, true>), dim3(p.nwg * p.nch), dim3(kThreads), 0, c.stream, m);
        else
          hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, NH, 0, K, true>), dim3(p.nwg * p.nch), dim3(64 * tile_waves(RT)), 0,
                             c.stream, m);
        return;
      }
    }
    if constexpr (NH > 2) {
      hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, NH, 0, 0>), dim3(p.nwg * p.nch), dim3(64 * tile_waves(RT)), 0, c.stream,
                         m);
    } else {
      by_cp([&](auto cpc) {
        constexpr int CP = decltype(cpc)::value;
        if constexpr (RT == 16 && NH == 1)
          hipLaunchKernelGGL((fused_dense_mfma_r16<LOSS, CP, K>), dim3(p.nwg * p.nch), dim3(kThreads), 0, c.stream, m);
        else
          hipLaunchKernelGGL((fused_dense_mfma<LOSS, RT, NH, CP, K>), dim3(p.nwg * p.nch), dim3(64 * tile_waves(RT)), 0,
                             c.stream, m);
      });
    }
  };
  if constexpr (NH > 2) {
    go(std::integral_constant<int, 0>{});
  } else {
    switch (nk) {
      case 1: go(std::integral_constant<int, 1>{}); break;
      case 2: go(std::integral_constant<int, 2>{}); break;
      case 3: go(std::integral_constant<int, 3>{}); break;
      default: go(std::integral_constant<int, 4>{}); break;
    }
  }
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



template <int LOSS, int RT, int NH, int DMA16, int PK = 1>
void launch_batch_variant(const BatchRun& b, int v, int want, hipStream_t st) {
  const dim3 grid((unsigned)b.vgrid[v]);
  if constexpr (RT == 16 && NH == 1)
    hipLaunchKernelGGL((batch_grad_kernel_r16<LOSS, DMA16, PK>), grid, dim3(kThreads), 0, st, b.desc, b.state,
                       b.items, b.vbegin[v], b.vend[v], b.counter + v, want);
  else
    hipLaunchKernelGGL((batch_grad_kernel<LOSS, RT, NH, DMA16, PK>), grid, dim3(kThreads), 0, st, b.desc, b.state,
                       b.items, b.vbegin[v], b.vend[v], b.counter + v, want);
}

// variant v = loss * 12 + (R > 16) * 6 + mode * 2 + (copy mode 2), mode 0:
// one h-tile, 1: two h-tiles, 2: one h-tile with two pairs per step
// (windows of at most 7 slots)
template <int LOSS>
void launch_batch_loss(const BatchRun& b, int v, int want, hipStream_t st) {
  switch (v % 12) {
    case 0: launch_batch_variant<LOSS, 16, 1, 1>(b, v, want, st); break;
    case 1: launch_batch_variant<LOSS, 16, 1, 2>(b, v, want, st); break;
    case 2: launch_batch_variant<LOSS, 16, 2, 1>(b, v, want, st); break;
    case 3: launch_batch_variant<LOSS, 16, 2, 2>(b, v, want, st); break;
    case 4: launch_batch_variant<LOSS, 16, 1, 1, 2>(b, v, want, st); break;
    case 5: launch_batch_variant<LOSS, 16, 1, 2, 2>(b, v, want, st); break;
    case 6: launch_batch_variant<LOSS, 32, 1, 1>(b, v, want, st); break;
    case 7: launch_batch_variant<LOSS, 32, 1, 2>(b, v, want, st); break;
    case 8: launch_batch_variant<LOSS, 32, 2, 1>(b, v, want, st); break;
    case 9: launch_batch_variant<LOSS, 32, 2, 2>(b, v, want, st); break;
    case 10: launch_batch_variant<LOSS, 32, 1, 1, 2>(b, v, want, st); break;
    default: launch_batch_variant<LOSS, 32, 1, 2, 2>(b, v, want, st); break;
  }
}

}  // namespace
}  // namespace gcp
