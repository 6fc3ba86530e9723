// Internal interfaces between the C-ABI shell (abi.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gcp {

constexpr int kMaxNs = 65;        // current slice + window of at most 64
constexpr int kMaxRank = 64;

enum Loss { kGaussian = 0, kPoissonLog = 1, kBernoulliLogit = 2, kPoissonId = 3, kBernoulliOdds = 4,
            // internal: the Gaussian gradient without the model (y = -2x); the
            // model's part is added from Gram matrices
            kGaussianId = 5 };
// epsilon of log(m + eps) in the identity- and odds-link losses (m >= 0)
constexpr double kLossEps = 1e-10;
// kWantObjective (with kWantLoss): the objective of the factor solve, in
// which s_t is fixed, so the mu/2 ||s_t||^2 term is left out
enum Want { kWantLoss = 1, kWantGrad = 2, kWantObjective = 4 };

// Deferred device status bits (workspace word).
enum StatusBits { kStatusNonFinite = 1, kStatusPivot = 2, kStatusSampler = 4 };

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Elementwise loss and derivative (Section 2.2 with log / logit links).
template <typename T, int LOSS>
struct LossFn;

template <typename T>
struct LossFn<T, kGaussian> {
  __device__ __forceinline__ static void eval(T x, T m, T& f, T& y) {
    T d = m - x;
    f = d * d;
    y = d + d;
  }
};

template <typename T>
struct LossFn<T, kPoissonLog> {
  __device__ __forceinline__ static void eval(T x, T m, T& f, T& y) {
    T e = exp(m);
    f = e - x * m;
    y = e - x;
  }
};

template <typename T>
struct LossFn<T, kBernoulliLogit> {
  __device__ __forceinline__ static void eval(T x, T m, T& f, T& y) {
    // log(1+e^m) = max(m,0) + log1p(e^-|m|); sigmoid from the same e^-|m|
    T e = exp(-fabs(m));
    T inv = T(1) / (T(1) + e);
    T sig = m >= T(0) ? inv : e * inv;
    f = fmax(m, T(0)) + log1p(e) - x * m;
    y = sig - x;
  }
};

template <typename T>
struct LossFn<T, kGaussianId> : LossFn<T, kGaussian> {};

template <typename T>
struct LossFn<T, kPoissonId> {
  __device__ __forceinline__ static void eval(T x, T m, T& f, T& y) {
    const T me = m + T(kLossEps);
    f = m - x * log(me);
    y = T(1) - x / me;
  }
};

template <typename T>
struct LossFn<T, kBernoulliOdds> {
  __device__ __forceinline__ static void eval(T x, T m, T& f, T& y) {
    const T me = m + T(kLossEps);
    f = log1p(m) - x * log(me);
    y = T(1) / (m + T(1)) - x / me;
  }
};

// FP32 loss evaluation on the hardware exp/log units (__expf, __logf: a few
// ulp), for kernels where the loss is the dominant vector-ALU cost.  The
// derivative is always formed; the loss value only when asked.
template <int LOSS>
struct LossFast;

template <>
struct LossFast<kGaussian> {
  __device__ __forceinline__ static float y(float x, float m) { return 2.f * (m - x); }
  __device__ __forceinline__ static float f(float x, float m) { return (x - m) * (x - m); }
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) {
    const float d = m - x;
    f = d * d;
    y = 2.f * d;
  }
};

template <>
struct LossFast<kPoissonLog> {
  __device__ __forceinline__ static float y(float x, float m) { return __expf(m) - x; }
  __device__ __forceinline__ static float f(float x, float m) { return __expf(m) - x * m; }
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) {
    const float e = __expf(m);
    f = e - x * m;
    y = e - x;
  }
};

template <>
struct LossFast<kBernoulliLogit> {
  __device__ __forceinline__ static float y(float x, float m) {
    const float e = __expf(-fabsf(m));
    const float inv = __frcp_rn(1.f + e);
    return (m >= 0.f ? inv : e * inv) - x;
  }
  __device__ __forceinline__ static float f(float x, float m) {
    return fmaxf(m, 0.f) + __logf(1.f + __expf(-fabsf(m))) - x * m;
  }
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) {
    const float e = __expf(-fabsf(m));
    const float inv = __frcp_rn(1.f + e);
    f = fmaxf(m, 0.f) + __logf(1.f + e) - x * m;
    y = (m >= 0.f ? inv : e * inv) - x;
  }
};

template <>
struct LossFast<kPoissonId> {
  __device__ __forceinline__ static float y(float x, float m) { return 1.f - x * __frcp_rn(m + (float)kLossEps); }
  __device__ __forceinline__ static float f(float x, float m) { return m - x * __logf(m + (float)kLossEps); }
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) {
    const float me = m + (float)kLossEps;
    f = m - x * __logf(me);
    y = 1.f - x * __frcp_rn(me);
  }
};

template <>
struct LossFast<kBernoulliOdds> {
  __device__ __forceinline__ static float y(float x, float m) {
    return __frcp_rn(m + 1.f) - x * __frcp_rn(m + (float)kLossEps);
  }
  __device__ __forceinline__ static float f(float x, float m) {
    return __logf(m + 1.f) - x * __logf(m + (float)kLossEps);
  }
  __device__ __forceinline__ static void fy(float x, float m, float& f, float& y) {
    const float me = m + (float)kLossEps;
    f = __logf(m + 1.f) - x * __logf(me);
    y = __frcp_rn(m + 1.f) - x * __frcp_rn(me);
  }
};

// Kahan-compensated accumulation.
template <typename T>
struct Kahan {
  T s = 0, c = 0;
  __device__ __forceinline__ void add(T v) {
    T yv = v - c;
    T t = s + yv;
    c = (t - s) - yv;
    s = t;
  }
};

// Fixed-order reduction of partial slots (used by the single-stream and the
// batched reduce kernels): a workgroup of 256 threads takes kRedOut outputs
// and splits their slots into kRedChunks fixed chunks.
constexpr int kRedOut = 16;     // outputs per workgroup
constexpr int kRedChunks = 16;  // slot chunks per output
constexpr int kRedUnroll = 8;   // loads in flight per thread

// k += f(p[i]) for i = begin, begin + step, ... < end, in that order; the
// loads of kRedUnroll consecutive terms are issued before their additions.
template <typename T, typename F>
__device__ __forceinline__ void kahan_strided(Kahan<T>& k, const T* p, size_t begin, size_t end, size_t step,
                                              F f) {
  for (size_t i = begin; i < end; i += kRedUnroll * step) {
    T v[kRedUnroll];
#pragma unroll
    for (int u = 0; u < kRedUnroll; ++u) {
      const size_t j = i + u * step;
      v[u] = j < end ? p[j] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kRedUnroll; ++u)
      if (i + u * step < end) k.add(f(v[u]));
  }
}

// ---------------------------------------------------------------------------
// Dense fused objective / gradient over the current slice and the window.
struct DenseCall {
  int I1, I2, I3, R;
  int ns;                       // 1 + number of window slices
  int loss;
  int want;
  int dtype;                    // 0 = f32, 1 = f64
  const void* X[kMaxNs];        // slice h (0 = current)
  const void* ring;             // window ring: slice h >= 1 is slot h-1 at ring + (h-1)*ring_stride
  const void* shist;            // window weights: s_h at shist + (h-1)*R
  size_t omega;                 // I1 I2 I3
  size_t ring_pitch;            // row pitch of stored slices (>= I3; X[0] has pitch I3)
  size_t ring_stride;           // elements per stored slice (I1 I2 ring_pitch)
  const void* S[kMaxNs];        // weight row of slice h (R values)
  double c[kMaxNs];             // c_0 = 1, c_h = w theta^(t-h)
  const void* A[3];
  void* G[3];
  void* gs;
  void* loss_out;
  double lam, mu;
  void* part;                   // partial-sum scratch (workspace)
  size_t part_bytes;
  int* status;
  hipStream_t stream;
  hipEvent_t ev_begin;          // optional: recorded around the main kernel
  hipEvent_t ev_end;
  int kernel;                   // 0 automatic, 1 VALU kernel, 2 matrix-core kernel
  int plan_target;              // matrix-core work plan (wanted wave blocks)
  const void* grad_scale;       // optional device scalar multiplying the gradients
  int xbits;                    // slices bit-packed (binary data; rows of ceil(I3/32) words)
  int merged34;                 // the third mode is modes 3 and 4 merged: no regulariser on it here
};

// Matrix-core (MFMA) variant of the fused kernel: work plan and launcher.
struct MfmaPlan {
  int tb1, tb2, nb1, nb2, nblocks, nwg;
  // I3 chunks (whole 32-entry groups, gpc per chunk): a single stream whose
  // pair tiles fill few compute units gives each (tile, chunk) a workgroup
  // of its own; the launch has nwg * nch workgroups
  int nch = 1, gpc = 1 << 30;
};
bool mfma_supported(int R, int ns, int dtype);
// target: wanted number of wave blocks (0 = default).  Candidates the
// autotuner tries are kPlanTargets; workspaces are sized for all of them.
constexpr int kPlanTargets[] = {256, 512, 1024, 2048, 4096, 8192, 16384};
constexpr int kNumPlanTargets = 7;
constexpr int kDefaultPlanTarget = 4096;
// Default plan of a stream's share of a batched call: fewer, larger blocks
// than a single stream's (the other streams supply the parallelism, and
// fewer workgroups write fewer partial sums): the 64-stream C4 step took
// 8.1 ms at 1024 against 8.4 at 512, 8.4 at 2048 and 9.1 at 4096.
constexpr int kBatchPlanTarget = 1024;
// Waves per workgroup of the matrix-core tile builds.  A single stream's
// rank-32 builds take four: their LDS allows one eight-wave workgroup per
// compute unit, but two or three four-wave ones, and one that finishes is
// replaced while the others keep the unit busy.  Rank 16 and the batched
// builds (whose work list already keeps every unit fed) take eight.
constexpr int kBatchTileWaves = 8;
constexpr int single_tile_waves(int R) { return R > 16 ? 4 : 8; }
// waves: waves per workgroup of the launch the plan is for
MfmaPlan mfma_plan(int I1, int I2, int I3, int waves, int target = kDefaultPlanTarget, bool chunk_i3 = false);
// Plan target of a single stream's call when none was tuned (a stream's
// plan_target of 0): the candidate whose workgroups fill their last round
// of resident workgroups best.
int auto_plan_target(int I1, int I2, int I3, int R, int ns);
hipError_t dense_mfma_launch(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                             float* gsp, float* lossp);
// Per-loss instantiations of the matrix-core tile code (one translation unit
// each): the single-stream launch and one batched variant launch.
hipError_t dense_mfma_launch_gaussian(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                      float* gsp, float* lossp);
hipError_t dense_mfma_launch_poisson(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                     float* gsp, float* lossp);
hipError_t dense_mfma_launch_gaussian_id(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p,
                                         float* G3p, float* gsp, float* lossp);
hipError_t dense_mfma_launch_poisson_id(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                        float* gsp, float* lossp);
hipError_t dense_mfma_launch_bernoulli_odds(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p,
                                            float* G3p, float* gsp, float* lossp);
hipError_t dense_mfma_launch_bernoulli(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                       float* gsp, float* lossp);
struct BatchRun;
void batch_launch_gaussian(const BatchRun& b, int v, int want, hipStream_t st);
void batch_launch_poisson(const BatchRun& b, int v, int want, hipStream_t st);
void batch_launch_bernoulli(const BatchRun& b, int v, int want, hipStream_t st);

size_t dense_fused_part_bytes(int I1, int I2, int I3, int R, int dtype);
hipError_t dense_fused_run(const DenseCall& c);

// Single-slice matrix-core kernel (no stored window): 4 x 4 blocks of
// (i1, i2) pairs per wave; partial slots G1: nb2, G2: nb1, G3 / g_s / loss: nwg.
struct SsPlan {
  int nb1, nb2, nblocks, nwg;
};
SsPlan single_slice_plan(int I1, int I2);
bool single_slice_supported(const DenseCall& c);
hipError_t single_slice_launch(const DenseCall& c, float* G1p, float* G2p, float* G3p, float* gsp, float* lossp);

// Batched multi-stream path (dense FP32, matrix-core tiles).
struct FacState;
struct BatchDesc {                 // per stream, fixed at batch creation
  const float* Xt;                 // registered input buffers
  const float* st;
  float* ring;                     // the stream's own workspace
  float* shist;
  float* A;
  float* Aold;
  float* u;
  float* v;
  float* Gs;
  float* G1p;                      // partial slots (batch workspace)
  float* G2p;
  float* G3p;
  float* gsp;
  float* lossp;
  float* outG[3];                  // where the reduce writes
  float* outgs;
  float* outloss;
  int64_t omega, fac_elems, fac_off1, fac_off2;
  int64_t rp3, rstride;          // row pitch / slot stride of the stored slices
  int I1, I2, I3, R, H, loss, variant;
  int tb1, tb2, nb1, nb2, nblocks, nwg;
  float lam, mu, lower, beta1, beta2, eps;
  double w, theta, alpha, beta1d, beta2d;   // history weights and ADAM rate in FP64
  uint64_t seed;
  // epochs of the factor solve (kappa_f > 0): the stream's solver state and
  // its saved copies of A, u, v (null without epochs)
  FacState* fac;
  float* Ao;
  float* uo;
  float* vo;
  double tol_f;
};
struct BatchState {                // per stream, advanced on the device
  int64_t t;
  int64_t adam_i;
  int nwin;
  int pending_slot;
  int64_t slot_t[kMaxNs];
};
// Copy mode of the matrix-core kernels' staged slice rows, for stored rows
// of pitch `pitch` values and a current slice of row length I3: rows are
// copied to LDS 16 bytes at a time when they are 16-byte aligned and their
// byte pitch fits 32 bits (the copy address is one 32 x 32 -> 64-bit
// multiply-add).  2: every row so (I3 a multiple of 4); 1: the stored rows
// so and the current slice's rows by 4-byte copies of their own; 0: 4-byte
// copies only.  A stream's window rows are padded to 32 values, so its
// stored rows always qualify.
inline int copy_mode(size_t pitch, int I3) {
  if (pitch % 4 != 0 || pitch >= ((size_t)1 << 29)) return 0;
  return I3 % 4 == 0 ? 2 : 1;
}

// Variants of the batched tile code: loss x (rank tile 16/32) x (one h-tile,
// two h-tiles, or one h-tile with two pairs per step for windows of at
// most 7 slots) x (16- or 4-byte slice-row copies), index
// loss * 12 + (R > 16) * 6 + mode * 2 + (copy mode 2 ? 1 : 0); batched
// streams take copy mode 1 or 2.
constexpr int kBatchVariants = 36;

constexpr int kBatchLanes = 4;   // HIP streams the variant launches are spread over
struct BatchRun {
  const BatchDesc* desc;
  BatchState* state;
  const int2* items;        // work list grouped by variant
  int nitems;
  int vbegin[kBatchVariants], vend[kBatchVariants];  // each variant's items
  int vgrid[kBatchVariants];                         // persistent workgroups per variant
  int vorder[kBatchVariants];  // the variants present, most expensive first
  int vlane[kBatchVariants];   // lane (HIP stream) of each variant
  int nvar, nlanes;
  hipStream_t lane[kBatchLanes];   // lane 0 is `stream`; the others belong to the batch
  hipEvent_t fork, join[kBatchLanes];
  int* counter;             // kBatchVariants work counters
  int nstreams;
  const int64_t* outstart;
  int64_t nout;
  const int64_t* facstart;
  int64_t nfac;
  const int64_t* cpystart;
  int64_t ncpy;
  int* status;
  hipStream_t stream;
};
int batch_variant(int loss, int R, int H, size_t pitch, int I3);
// Whether variant v runs two workgroups per compute unit.
bool batch_variant_r16(int v);
hipError_t batch_grad_run(const BatchRun& b, int want);
hipError_t batch_adam_run(const BatchRun& b);
hipError_t batch_window_run(const BatchRun& b);
// Algorithm 4's epochs for every stream of a batch, decided on the device:
// begin (objective at the start), one ADAM step with the device-held rate,
// end of epoch (keep or undo).  The objective is the one the last
// batch_grad_run(kWantLoss | kWantObjective) wrote to the step descriptors.
hipError_t batch_fac_begin_run(const BatchRun& b);
hipError_t batch_fac_step_run(const BatchRun& b);
hipError_t batch_fac_end_run(const BatchRun& b, int tau_f);

// Stratified sampled objective/gradient over COO slices (FP32).
struct SampledCall {
  int I1, I2, I3, R, ns, loss, want;
  const int32_t* coords[kMaxNs];  // nnz x 3, sorted by row-major linear index
  const void* vals[kMaxNs];
  const uint64_t* tab[kMaxNs];    // membership table of slice h (table_build)
  uint64_t tab_cap;               // capacity of every table
  int64_t nnz[kMaxNs];
  int64_t stamp[kMaxNs];          // time stamp of slice h (sampler counter word)
  const void* S[kMaxNs];
  double c[kMaxNs];
  const void* A[3];
  void* G[3];
  void* gs;
  void* loss_out;
  double lam, mu;
  int64_t p, q;
  uint64_t seed;
  int64_t call;                   // sampler call number
  int* status;
  hipStream_t stream;
  hipEvent_t ev_begin, ev_end;
  // Row-sorted reduction (null srec: one float atomic per draw, row and
  // rank column instead).  srec: one 16-byte record per draw slot
  // (ns x ceil((p+q)/64) x 64); ssrt: three lists of ns (p+q) 16-byte
  // records; scnt: per mode I_k counts, I_k + 1 row starts and I_k cursors;
  // sS: ns x R weight rows.
  void* srec;
  void* ssrt;
  int* scnt;
  float* sS;
};
// Model-difference history term (eq. gcp_stream_problem_2): adds
// 1/2 sum_h w_h ||[[Abar; s_h]] - [[A; s_h]]||^2 to *loss and its factor
// gradient (times *grad_scale) to G, after the data term has written them.
struct HistCall {
  int I[3], R, nwin, dtype, want;
  const void* A[3];
  const void* Ab[3];        // previous step's factors
  const void* shist;        // nwin x R stored weights
  const int64_t* stamps;    // device, time stamp t_h of each window slot (nwin values)
  int64_t t;                // current time: w_h = w theta^(t - t_h)
  double w, theta;
  void* G[3];
  void* loss;
  const void* grad_scale;
  double* ws;               // hist_ws_bytes(R)
  int* status;
  hipStream_t stream;
};
size_t hist_ws_bytes(int R);
hipError_t hist_run(const HistCall& c);
// One device-held slot stamp update (a window push).
hipError_t hist_set_stamp_run(int64_t* stamps, int slot, int64_t t, hipStream_t stream);
constexpr int kMaxWindowModel = 4096;   // GCP_MAX_WINDOW_MODEL
// Gaussian gradient through the identity of Section 5: after a data pass
// with y = -2x, adds the model's part G_k += 2 A_k ((*_{l != k} A_l'A_l) o S),
// S = s_t s_t' + sum_h c_h s_h s_h' (c.shist, c.c over c.nwin slots), and
// g_s += 2 (*_l A_l'A_l) s_t.  Uses c.A, c.G, c.ws, c.R, c.I, c.dtype.
hipError_t ident_run(const HistCall& c, const void* s_t, void* g_s);

// Workspace bytes of the row-sorted reduction for a stream (0: not used).
size_t sampled_sorted_bytes(int I1, int I2, int I3, int R, int window, int64_t p, int64_t q);
// Point c's row-sorted buffers into a workspace of sampled_sorted_bytes bytes
// (c's sizes, p and q must be set).
void sampled_sorted_bind(SampledCall& c, char* base, int window);
// Membership table of a COO slice: capacity for up to max_nnz entries, and
// the build (fill + insert, two launches on `stream`).
uint64_t table_capacity(int64_t max_nnz);
hipError_t table_build(const int32_t* coords, int64_t nnz, int I2, int I3, uint64_t* tab, uint64_t cap,
                       hipStream_t stream);
hipError_t sampled_run(const SampledCall& c);
// Writes the draws of slice h of c (coordinates, weights) as sampled_run forms them.
hipError_t sampled_dump_run(const SampledCall& c, int h, int32_t* coords, float* weights);

// Unfused baseline: model, elementwise, per-mode MTTKRP kernels.
size_t dense_plain_scratch_bytes(int I1, int I2, int I3, int R, int dtype);
hipError_t dense_plain_run(const DenseCall& c, void* scratch, size_t scratch_bytes);
// Gather roof probe of the sampled path (measurement only).
hipError_t gather_probe_run(const float* A1, const float* A2, const float* A3, int I1, int I2, int I3, int R,
                            int64_t ndraws, uint64_t seed, void* rec, hipStream_t st);

// Least-squares temporal solve (FP64 normal equations).
size_t ls_scratch_bytes(int I1, int I2, int I3, int R);
hipError_t ls_solve_run(int I1, int I2, int I3, int R, int dtype, const void* X,
                        const void* const* A, double mu, double lower, void* s_out,
                        void* scratch, int* status, hipStream_t st);

// ADAM step over a flat array (Algorithm 2, Step).
hipError_t adam_run(int dtype, int64_t n, void* a, const void* g, void* u, void* v,
                    double alpha_t, double beta1, double beta2, double eps,
                    double lower, hipStream_t st);

}  // namespace gcp
