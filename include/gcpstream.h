/*
 * gcpstream: streaming generalized CP (GCP) objective and gradient on one
 * MI355X (gfx950).  C ABI.
 *
 * The method is OnlineGCP (Phipps, Johnson, Kolda, "Streaming Generalized
 * Canonical Polyadic Tensor Decompositions").  At time step t the library
 * evaluates, over the current d-way slice X_t and a window H_t of stored past
 * slices X_h (Section 4.1, eq. gcp_stream_problem_1),
 *
 *   F = sum_i f(x_it, m_i(s_t)) + sum_{h in H_t} w_h sum_i f(x_ih, m_i(s_h))
 *       + lambda/2 sum_k ||A^(k)||_F^2 + mu/2 ||s_t||^2,
 *   m_i(s) = sum_j s_j prod_k A^(k)[i_k, j]        (eq. CP_model)
 *   w_h = w theta^(t-h)                             (Section 4.1)
 *
 * and its gradients (eqs. gcp_grad_A, gcp_grad_lambda, Section 4.2)
 *
 *   G^(k) = Y_t(k) Z_k diag(s_t) + sum_h w_h Y_h(k) Z_k diag(s_h) + lambda A^(k)
 *   g_s   = Z^T vec(Y_t) + mu s_t,        y_i = df/dm (x_i, m_i).
 *
 * Losses: Gaussian f = (x-m)^2; Poisson with log link f = e^m - x m;
 * Bernoulli with logit link f = log(1+e^m) - x m (Section 2.2 with the
 * m-independent terms dropped).
 *
 * Conventions shared by every call
 *  - Slices of order d = 3, or d = 2 (matrix slices; GCP_E_UNSUPPORTED otherwise).
 *  - A dense slice is I_1 x I_2 x I_3, row-major (last index contiguous),
 *    base aligned to 16 bytes.  A factor matrix A^(k) is I_k x R row-major.
 *  - Every array argument is a DEVICE pointer unless marked "host".
 *  - The library never allocates or frees device memory: the caller passes
 *    one workspace of gcp_workspace_size() bytes (256-byte aligned) that the
 *    stream owns until gcp_stream_destroy.  The handle lives on the host heap.
 *  - Every call is asynchronous on the HIP stream given at init and performs
 *    no host synchronisation, except where documented (gcp_stream_sync and
 *    the sample dump).  A handle is not thread-safe.
 *  - Argument, shape, alignment and state errors are detected before any
 *    launch and leave the stream unchanged.  Device-detected numeric failures
 *    (non-finite loss or gradient, a failed Cholesky pivot) set a status word
 *    in the workspace that gcp_stream_sync returns (GCP_E_NUMERIC).
 *  - Outputs are overwritten, never accumulated into.
 */
#ifndef GCPSTREAM_H
#define GCPSTREAM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCP_ABI_VERSION 2
#define GCP_MAX_D 4
#define GCP_MAX_RANK 64
#define GCP_MAX_WINDOW 64          /* stored-slice history */
#define GCP_MAX_WINDOW_MODEL 4096  /* model-difference history (weights only) */
/* Size of the library's fixed per-GPU device array used by
 * gcp_loss_grad_static (64 MiB). */
#define GCP_STATIC_SCRATCH_BYTES (64u << 20)

typedef struct gcp_stream gcp_stream;

typedef enum {
  GCP_OK = 0,
  GCP_E_ARG = 1,          /* bad scalar argument or null pointer          */
  GCP_E_SHAPE = 2,        /* dimension / size mismatch                     */
  GCP_E_ALIGN = 3,        /* misaligned dense base or workspace            */
  GCP_E_STATE = 4,        /* call not valid in the stream's current state  */
  GCP_E_WORKSPACE = 5,    /* workspace too small                           */
  GCP_E_DEVICE = 6,       /* a HIP runtime call failed                     */
  GCP_E_NUMERIC = 7,      /* device found a non-finite value / bad pivot   */
  GCP_E_UNSUPPORTED = 8   /* valid request outside what is implemented     */
} gcp_status;

typedef enum {
  GCP_LOSS_GAUSSIAN = 0,
  GCP_LOSS_POISSON_LOG = 1,
  GCP_LOSS_BERNOULLI_LOGIT = 2,
  /* The two losses Section 2.2 writes out, for m >= 0 (take lower = 0):
   * count data, identity link: f = m - x log(m + eps), eps = 1e-10;
   * binary data, odds link:    f = log(m + 1) - x log(m + eps).
   * Dense and COO single streams (not in batches); no LS solve. */
  GCP_LOSS_POISSON_ID = 3,
  GCP_LOSS_BERNOULLI_ODDS = 4
} gcp_loss;

typedef enum { GCP_F32 = 0, GCP_F64 = 1 } gcp_dtype;
/* Slice storage.  BITS: a dense binary slice (the binary data of Section
 * 2.2) packed one bit per entry: each (i1, i2) row of I3 entries takes
 * ceil(I3 / 32) 32-bit words, entry i3 is bit i3 % 32 (least significant
 * first) of word i3 / 32; bits past I3 are ignored.  Window slots keep the
 * same layout, so a stored slice takes 1/32 of the FP32 bytes.  BITS streams:
 * Bernoulli losses, GCP_F32, d = 3, window <= 31, rank <= 32, the
 * stored-slice history, not GCP_FLAG_KERNEL_VALU, no batches. */
typedef enum { GCP_SLICE_DENSE = 0, GCP_SLICE_COO = 1, GCP_SLICE_BITS = 2 } gcp_slice_kind;

/* Bits of the `want` argument of gcp_loss_grad. */
enum {
  GCP_WANT_LOSS = 1,      /* write *loss                                  */
  GCP_WANT_GRAD = 2,      /* write G^(1..d) and g_s                       */
  GCP_IMPL_PLAIN = 256    /* run the unfused multi-kernel path instead    */
};

/* History term of the objective (gcp_params.hist), Section 4.1.
 * SLICES: the window stores past slices X_h with their weights s_h and adds
 *   sum_h w_h sum_i f(x_ih, m_i(s_h)) (eq. gcp_stream_problem_1).
 * MODEL: the window stores only the weights s_h and adds
 *   1/2 sum_h w_h ||[[Abar; s_h]] - [[A; s_h]]||_F^2 (eq. gcp_stream_problem_2),
 *   Abar being the factors at the end of the previous time step (at stream
 *   creation: A0); the data term is that of X_t alone, and the factor
 *   gradient gains A_k B_k - Abar_k C_k (eq. spatial_gcp_grad), evaluated
 *   through R x R Gram matrices in FP64.  No window slice is stored, so the
 *   workspace holds no slice ring. */
typedef enum { GCP_HIST_SLICES = 0, GCP_HIST_MODEL = 1 } gcp_hist;

/* Temporal-weight solver of gcp_solve_st (gcp_params.tsolve).
 * LS: the least-squares solve of Section 5 (Gaussian loss only).
 * SGD: Algorithm 3, any loss: s <- 0 and fresh ADAM moments,
 *   then at most kappa_w epochs while F > tol_w, each tau_w ADAM steps
 *   (Algorithm 2, Step, rate alpha_w, iteration index i from 0) on the
 *   gradient of F(s) = sum_i f(x_i, m_i(s)) + mu/2 ||s||^2 over X_t, then
 *   F at the new s; an epoch that raised F is rolled back (s and the moments
 *   return to the last accepted epoch, i goes back tau_w steps, the rate is
 *   multiplied by 0.1).  Dense slices: gradient and objective exact over
 *   X_t.  COO slices: each step's weight gradient is the sampled one of X_t
 *   alone (p nonzero and q zero draws, a new call number each), and F is
 *   Algorithm 5's estimate with p_est and q_est draws under the call number
 *   2^31 + 2^30 + (t mod 2^30), fixed for the solve. */
typedef enum { GCP_TSOLVE_LS = 0, GCP_TSOLVE_SGD = 1 } gcp_tsolve;

/* Flags of gcp_params.flags. */
enum {
  GCP_FLAG_PLAIN_SCRATCH = 1, /* reserve the unfused path's scratch (2 slices) */
  GCP_FLAG_KERNEL_VALU = 2,   /* fused path: always the vector-ALU kernel      */
  GCP_FLAG_KERNEL_MFMA = 4,   /* fused path: the matrix-core kernel wherever it
                                 applies (FP32, R <= 32, window <= 63);
                                 default: chosen by rank                     */
  GCP_FLAG_GAUSS_IDENTITY = 16, /* Gaussian dense streams: gradient-only calls
                                 (want = GCP_WANT_GRAD, no grad_scale, the
                                 fused path, every factor-update iteration)
                                 skip the model: with Y = 2(M - X), Section 5
                                 gives G_k = 2 A_k ((*_{l!=k} A_l'A_l) o S)
                                 - 2 X_(k) Z_k diag(s) summed over the slices
                                 (S = sum_h c_h s_h s_h'), so one pass forms
                                 the X term and FP64 Gram matrices the rest.
                                 The two terms cancel as the fit improves,
                                 so the FP32 result loses relative accuracy
                                 near a fit; objective calls are unchanged */
  GCP_FLAG_SAMPLED_ATOMIC = 8 /* COO gradient: one float atomic per draw, row
                                 and rank column instead of the row-sorted
                                 reduction (less workspace, slower; the
                                 sorted workspace is 64 (H+1)(p+q) bytes plus
                                 12 (I_1+I_2+I_3) and is reserved by default) */
};

/* Table 1 (Section 4.2) of the paper, plus layout and sampling controls. */
typedef struct {
  uint32_t abi_version;   /* GCP_ABI_VERSION                               */
  int32_t d;              /* slice order: 3, or 2 for matrix slices: dims
                           * (I1, I2, 1), slices I1 x I2 row-major, factors
                           * A^(1) (I1 x R) and A^(2) (I2 x R) in entries 0
                           * and 1 of every factor array (entry 2 unused,
                           * may be NULL).  Internally an I1 x 1 x I2
                           * tensor whose middle factor is a fixed row of
                           * ones (no ADAM steps, no regulariser; requires
                           * lower <= 1); COO coords are (i1, 0, i2).  No
                           * batches.
                           * Or 4 (the higher-order slices of Section 3.2):
                           * dims (I1, I2, I3, I4), dense slices
                           * I1 x I2 x I3 x I4 row-major, four factors in
                           * entries 0..3 of every factor and gradient
                           * array.  Evaluated with modes 3 and 4 merged:
                           * entry (i3, i4) is entry i3 I4 + i4 of an
                           * I1 x I2 x (I3 I4) slice (the same memory) whose
                           * third factor has the rows A3[i3] * A4[i4]
                           * (formed on the device each call); the merged
                           * mode's gradient projects onto A3 and A4 by the
                           * chain rule.  Dense slices only (FP32 or FP64),
                           * stored-slice history, I3 I4 <= 2^30; no COO,
                           * bit-packed slices, batches, GCP_FLAG_GAUSS_IDENTITY,
                           * GCP_FLAG_PLAIN_SCRATCH or autotuning.       */
  int64_t dims[GCP_MAX_D];/* I_1, I_2, I_3 (and I_4 when d = 4)           */
  int32_t rank;           /* R, 1..GCP_MAX_RANK                            */
  int32_t window;         /* H, 0..GCP_MAX_WINDOW (stored slices), or
                           * 0..GCP_MAX_WINDOW_MODEL with GCP_HIST_MODEL,
                           * which keeps only R weights per slot          */
  int32_t loss;           /* gcp_loss                                      */
  int32_t dtype;          /* gcp_dtype: GCP_F64 is for verification only  */
  int32_t slice_kind;     /* gcp_slice_kind of every slice of the stream  */
  int32_t flags;          /* GCP_FLAG_*                                    */
  double w, theta;        /* history weights w_h = w theta^(t-h)          */
  double lambda, mu;      /* factor / temporal-weight regularisation       */
  double lower;           /* lower bound l (-INFINITY: none)               */
  double alpha_f;         /* ADAM rate of the factor solver (Alg. 2)       */
  double beta1, beta2, adam_eps;
  int32_t tau_f;          /* factor iterations per gcp_update_factors      */
  int32_t hist;           /* gcp_hist: the history term of the objective   */
  int64_t max_nnz;        /* COO: largest nnz of any slice (X_t included);
                           * sizes the window slots and the per-slice
                           * membership tables (2 max_nnz keys of 8 B,
                           * rounded up to a power of 2)                  */
  int64_t p, q;           /* COO: nonzero / zero samples per gradient      */
  uint64_t seed;          /* reservoir draws and the sampler               */
  int32_t tsolve;         /* gcp_tsolve of gcp_solve_st                     */
  int32_t tau_w;          /* SGD: ADAM steps per epoch, >= 1                */
  int32_t kappa_w;        /* SGD: most epochs, 0..64                        */
  int32_t kappa_f;        /* factor epochs per gcp_update_factors, 0..64;
                           * 0: tau_f iterations, all kept (see there)     */
  double alpha_w;         /* SGD: initial ADAM rate, > 0                    */
  double tol_w;           /* SGD: stop once F <= tol_w (-INFINITY: never)   */
  double tol_f;           /* factor epochs: stop once F <= tol_f            */
  int64_t p_est, q_est;   /* COO streams with an SGD solver (kappa_f > 0 or
                           * GCP_TSOLVE_SGD): nonzero / zero draws per
                           * slice of Algorithm 5's objective estimate     */
} gcp_params;

/* One slice.  DENSE: vals holds prod(dims) values, coords is NULL.
 * COO: nnz entries; coords is nnz x 3 int32 row-major, sorted by row-major
 * linear index with no duplicates; vals are the (non-zero) values.
 * BITS: vals holds I1 I2 ceil(I3/32) uint32 words (4-byte aligned), coords
 * is NULL. */
typedef struct {
  int32_t kind;           /* gcp_slice_kind */
  int32_t reserved;
  const void* vals;       /* float or double, per gcp_params.dtype */
  const int32_t* coords;
  int64_t nnz;
} gcp_slice;

/* Fills *params with the paper's defaults (Table 2 caption, Section 6):
 * w = theta = 1, lambda = mu = 0, beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
 * lower = -inf, alpha_f = 1e-3, tau_f = 1, FP32, dense. */
void gcp_params_default(gcp_params* params);

/* Bytes of device workspace a stream with these parameters needs. */
gcp_status gcp_workspace_size(const gcp_params* params, size_t* bytes);

/* Creates a stream: the inputs of Algorithm 1 (Section 4.3) with the
 * arguments of Table 1 in params.  A0[k] (k < d) are the initial factor
 * matrices (the warm start); they and
 * the n_hist initial window slices X_hist[h] (host array of slice structs
 * whose data pointers are device pointers) with their weights s_hist
 * (device, n_hist x R) and host time stamps t_hist are COPIED into the
 * workspace, so the caller may free them after the stream has executed the
 * copies.  The stream's time index starts at max(t_hist)+1 (1 if empty).
 * n_hist must not exceed params->window.  With GCP_HIST_MODEL no slice is
 * kept: X_hist is ignored (it may be NULL) and the window is given by s_hist
 * and t_hist alone; A0 is also the first "previous-step" factors. */
gcp_status gcp_stream_init(const gcp_params* params, const void* const* A0,
                           int32_t n_hist, const gcp_slice* X_hist,
                           const void* s_hist, const int64_t* t_hist,
                           void* workspace, size_t ws_bytes,
                           hipStream_t hip_stream, gcp_stream** out);

/* Objective and gradient at (A, s_t) over X_t and the stream's window, with
 * the stream's current t for w_h (Section 4.2, eq. spatial_gcp_grad for the
 * stored-slice history).  A[k] may alias the stream's own factors
 * (gcp_factor_ptr).  want: GCP_WANT_LOSS and/or GCP_WANT_GRAD; add
 * GCP_IMPL_PLAIN for the unfused path (needs GCP_FLAG_PLAIN_SCRATCH).
 * loss: device scalar; G[k]: I_k x R; g_s: R.  Null outputs are allowed for
 * the parts not wanted.
 * COO streams (FP32): the data terms of every slice are the stratified
 * sampled estimates of Section 4.3 / Algorithm 6 with p nonzero and q zero
 * draws per slice and weights eta/p, zeta/q; the regularisation terms are
 * exact.  Draws use Philox4x32-10 with key = seed and counter = (draw number,
 * slice time stamp, call number, stratum + 2*attempt); the call number
 * starts at 0 and advances by one per sampled evaluation (including each
 * iteration of gcp_update_factors).  Zero draws are redrawn (at most 64
 * times, else GCP_E_NUMERIC) while they hit a stored entry.  The MTTKRP
 * rows are summed through row-sorted lists (GCP_FLAG_SAMPLED_ATOMIC: one
 * float atomic per draw and rank column); either way the order of the
 * additions varies, so the rounding does.
 * With GCP_HIST_MODEL the window term is the model difference of
 * eq. gcp_stream_problem_2 (see gcp_hist), added after the data term of X_t;
 * it uses the stream's previous-step factors and does not change g_s. */
gcp_status gcp_loss_grad(gcp_stream* s, const gcp_slice* X_t,
                         const void* const* A, const void* s_t, uint32_t want,
                         void* loss, void* const* G, void* g_s);

/* As gcp_loss_grad, with every gradient output multiplied on the device by
 * the scalar *grad_scale (device pointer, stream dtype; NULL means 1).  This
 * is the adjoint used by the differentiation wrapper: dL/dA^(k) =
 * grad_scale * G^(k), dL/ds_t = grad_scale * g_s, with the model recomputed
 * rather than stored.  The objective output is not scaled. */
gcp_status gcp_loss_grad_scaled(gcp_stream* s, const gcp_slice* X_t,
                                const void* const* A, const void* s_t,
                                uint32_t want, const void* grad_scale,
                                void* loss, void* const* G, void* g_s);

/* Temporal weights for X_t with the stream's factors held fixed (Alg. 1,
 * temporal step; eq. gcp_stream_temporal_problem), by params->tsolve:
 * GCP_TSOLVE_LS (Gaussian loss only): the least-squares solve of Section 5,
 *   (Gamma + mu/2 I) s = Z^T vec(X_t) with Gamma = hadamard_k A^(k)^T A^(k),
 *   formed and solved in FP64 on the device, then s <- max(s, l).
 * GCP_TSOLVE_SGD (any loss, dense or COO slices): Algorithm 3 as described
 *   at gcp_tsolve, every decision taken on the device (a fixed sequence of
 *   launches, no host synchronisation).  s_t is the solver's iterate while
 *   it runs.
 * Writes s_t (R values of the stream dtype). */
gcp_status gcp_solve_st(gcp_stream* s, const gcp_slice* X_t, void* s_t);

/* State of the last GCP_TSOLVE_SGD solve (waits for the HIP stream): the
 * objective at the returned weights, the final ADAM rate, the iteration
 * index, the epochs run, and a mask whose bit e is set when epoch e was
 * rolled back.  Any output may be NULL.  GCP_E_STATE for other solvers. */
gcp_status gcp_solve_st_info(gcp_stream* s, double* F, double* alpha, int64_t* iters, int32_t* epochs,
                             uint64_t* rolled);

/* Factor update for X_t with weights s_t (Alg. 1 factor step; Alg. 4):
 * kappa_f = 0: tau_f times [full gradient over X_t and the window, then the
 *   ADAM Step of Alg. 2 with the stream's global iteration index], every
 *   iteration kept.
 * kappa_f > 0: Alg. 4's epochs.  F = the objective without mu/2 ||s_t||^2:
 *   exact over X_t and the window for dense slices; for COO slices Alg. 5's
 *   estimate with p_est nonzero and q_est zero draws per slice, over draws
 *   fixed for the call (call number 2^31 + (t mod 2^30), apart from the
 *   gradients' counter) with exact history and regulariser terms; at most kappa_f epochs
 *   while F > tol_f, each tau_f [gradient, ADAM Step] iterations and then F
 *   at the new factors; an epoch that raised F is undone (factors and
 *   moments return to the last accepted epoch, the index goes back tau_f
 *   steps, the rate is multiplied by 0.1).  The rate, index and saved copies
 *   persist across calls (one ADAM object per stream, created with the
 *   stream; the saved factors start as A0).  Every decision is taken on the
 *   device: no host synchronisation.
 * Then A_old <- A, the reservoir window update with X_t and s_t, and
 * t <- t+1.  X_t may be reused by the caller once the HIP stream has passed
 * this call. */
gcp_status gcp_update_factors(gcp_stream* s, const gcp_slice* X_t,
                              const void* s_t);

/* State of the factor epochs of the last gcp_update_factors (waits for the
 * HIP stream): the objective at the accepted factors, the current ADAM rate,
 * the iteration index, the epochs run and the mask of rolled-back epochs.
 * Any output may be NULL.  GCP_E_STATE when params->kappa_f is 0. */
gcp_status gcp_factor_info(gcp_stream* s, double* F, double* alpha, int64_t* iters, int32_t* epochs,
                           uint64_t* rolled);

/* Reconstruction loss of a dense slice X (Section 6, eq. local_loss) under
 * the CP model of the stream's current factors with weights s_x (device, R
 * values): *sum_f = sum_i f(x_i, m_i) (no history or regularisation terms),
 * *sum_sq = ||X||_F^2, both host doubles (the call waits for the stream).
 * The local loss is sum_f / sum_sq for the current slice; the global loss of
 * Section 6 is the ratio of the sums over all past slices with the final
 * factors.  Dense streams only (GCP_E_UNSUPPORTED for COO). */
gcp_status gcp_slice_loss(gcp_stream* s, const gcp_slice* X, const void* s_x, double* sum_f, double* sum_sq);

/* Local reconstruction loss of Section 6, eq. local_loss: sum_f / sum_sq of
 * gcp_slice_loss for the dense slice X with weights s_x under the stream's
 * current factors, written to *out (host double; the call waits for the
 * stream).  *out is NaN when ||X||_F = 0 (the ratio is undefined).  Dense
 * streams only (GCP_E_UNSUPPORTED for COO). */
gcp_status gcp_local_loss(gcp_stream* s, const gcp_slice* X, const void* s_x, double* out);

/* K-tensor score of Section 6.1 (congruence of the computed and a reference
 * K-tensor, 1.0 for a perfect recovery): the stream's current factors with
 * component weights w_a (device, R values) against B[k] (device, I_k x
 * rank_b row-major) with weights w_b (device, rank_b values), all of the
 * stream dtype.  Columns are normalised with their norms moved into the
 * weights; a pair (r, q) scores (1 - |xi_r - eta_q| / max(xi_r, eta_q)) times
 * the product over modes of |cos(a_r, b_q)|; pairs are matched greedily
 * (highest first, each component once) and *score (host) is the sum of the
 * matched pair scores over rank_b.  Waits for the stream. */
gcp_status gcp_ktensor_score(gcp_stream* s, const void* w_a, const void* const* B, const void* w_b, int32_t rank_b,
                             double* score);

/* Copies the stream's current factors into A_out[k] (device, k < d). */
gcp_status gcp_get_factors(gcp_stream* s, void* const* A_out);

/* Device pointer to the stream's current factor k < d (valid until destroy). */
gcp_status gcp_factor_ptr(gcp_stream* s, int32_t k, void** ptr);

/* Host-side stream state: current t, window size, Adam iteration index (with
 * kappa_f > 0 it is read from the device, which waits for the stream), the
 * time stamp held by each window slot (host array of params->window), and
 * the sampler's call number (COO streams: the number of sampled gradient
 * evaluations so far; the next one draws with this number).  Any output may
 * be NULL. */
gcp_status gcp_stream_info(gcp_stream* s, int64_t* t, int32_t* n_window,
                           int64_t* adam_iter, int64_t* slot_times,
                           int64_t* sample_call);

/* Waits for the HIP stream and returns the deferred device status
 * (GCP_E_NUMERIC if a kernel flagged one), clearing it. */
gcp_status gcp_stream_sync(gcp_stream* s);

gcp_status gcp_stream_destroy(gcp_stream* s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the dense
 * objective and gradients of gcp_loss_grad, with no stream handle and no
 * workspace.  The partial sums live in a fixed device array of
 * GCP_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; the call allocates nothing (no hipMalloc, no
 * library allocation) and only launches kernels on hip_stream.
 *   params: d = 3, dense, GCP_HIST_SLICES, FP32 or FP64 (dims, rank, loss,
 *           w, theta, lambda, mu and the kernel flags are used; no plain
 *           scratch or Gaussian-identity flag).
 *   X_t: dense slice (device, I1*I2*I3 row-major, 16-byte aligned).
 *   X_hist: device, n_hist slices of I1*I2*I3 values one after another
 *           (16-byte aligned; may be NULL when n_hist = 0), 0 <= n_hist <=
 *           params->window; s_hist: device n_hist x R weights; t_hist:
 *           host time stamps, each below t; t: the current time index, so
 *           slice h carries w theta^(t - t_hist[h]).
 *   A, s_t, want, loss, G, g_s: as for gcp_loss_grad (device pointers;
 *           outputs are overwritten).
 * Returns GCP_E_WORKSPACE when the partial sums of this shape do not fit
 * the array, the argument errors of gcp_loss_grad otherwise.  No
 * status word is reported: a non-finite result shows in the outputs.  Every
 * call on one GPU uses the same array, which keeps the last call's partial
 * sums (each call overwrites every slot it reads), so calls that overlap on
 * one GPU (on different HIP streams, or from different host threads) race
 * and must be serialised by the caller. */
gcp_status gcp_loss_grad_static(const gcp_params* params, const gcp_slice* X_t, int32_t n_hist,
                                const void* X_hist, const void* s_hist, const int64_t* t_hist, int64_t t,
                                const void* const* A, const void* s_t, uint32_t want, void* loss,
                                void* const* G, void* g_s, hipStream_t hip_stream);

/* Measurement tool, no part of the method: the sampled path's gather
 * pattern alone, to give it a measured roof.  For ndraws uniform random
 * (i1, i2, i3) (SplitMix64 of the draw number and seed), gathers the three
 * factor rows (device, I_k x rank row-major FP32) with the lane mapping of
 * the sampled gradient kernel, forms sum_j A1 A2 A3 and writes one 16-byte
 * record per draw to records (device, 16 ndraws bytes: the three indices as
 * int32 bits and the sum).  Asynchronous on hip_stream; time it with events. */
gcp_status gcp_probe_gather(const void* A1, const void* A2, const void* A3, int64_t I1, int64_t I2, int64_t I3,
                            int32_t rank, int64_t ndraws, uint64_t seed, void* records, hipStream_t hip_stream);

/* Autotuner for the matrix-core work plan of a stream's own calls (how the
 * slice's (i1,i2) pairs are cut into wave blocks: 256, 512, ..., 16384
 * blocks).  Untuned, a stream takes among 2048, 4096 and 8192 blocks the
 * plan whose workgroups fill their last round of resident workgroups best.
 * This call times every candidate plan on the device with HIP events over
 * X_t and the current window (synchronous; not for use inside a graph
 * capture): seven single calls per plan, taken round-robin over the plans;
 * it keeps the plan with the lowest median call for this stream (errors:
 * GCP_E_DEVICE when a device call fails), and appends "<key> = <plan>"
 * to the text file cache_path (NULL: no cache), where the key is the shape
 * bucket "<arch> loss<l> rt<16|32> nh<h-tiles> dma<copy mode 0|1|2>
 * pairs2^<floor(log2(I1 I2))> i3x64:<ceil(I3/64)>".  A cache hit (a valid
 * plan for the bucket) skips the timing.  Batched calls use the plan set by
 * gcp_batch_autotune instead.  Results are identical for every plan up to
 * summation order.  *chosen (may be NULL) receives the plan.  Dense FP32
 * streams only. */
gcp_status gcp_autotune(gcp_stream* s, const gcp_slice* X_t, const char* cache_path, int32_t* chosen);

/* ------------------------------------------------------------------------
 * Batching: many independent dense FP32 streams (rank <= 32, window <= 31)
 * advanced together.  Each stream keeps its own workspace; the batch adds a
 * workspace of gcp_batch_workspace_size() bytes with the stream descriptors,
 * work list, partial sums and the streams' device-side step state.
 * Per stream the caller registers fixed device buffers: X_t (dense slice)
 * and s_t (R weights) as inputs, and optional outputs for
 * gcp_batch_loss_grad (loss scalar, G[3], g_s; NULL: not written).  The
 * caller refreshes the input buffers' contents before each call.
 * All per-call state (time index, window fill and slot time stamps, ADAM
 * iteration, and with kappa_f > 0 the factor solver's rate, objective and
 * saved copies) is kept on the device, so any sequence of batch calls issued
 * on the batch's HIP stream may be captured once as a HIP graph and
 * replayed.  A single stream that fits these limits takes the same route as
 * a batch of one: its whole time step (gcp_batch_step) is then one graph.
 * While a stream is in a batch its host-side state (gcp_stream_info) is stale
 * until gcp_batch_sync_streams.  Outputs match the per-stream calls.
 * ------------------------------------------------------------------------ */
typedef struct gcp_batch gcp_batch;

typedef struct {
  const void* X_t;      /* device, I1*I2*I3 values, 16-byte aligned */
  const void* s_t;      /* device, R values                          */
  void* loss;           /* device scalar or NULL                     */
  void* G[3];           /* device I_k x R, or NULL                    */
  void* g_s;            /* device R, or NULL                          */
} gcp_batch_io;

/* Autotuning of a set of streams before they are batched (call it before
 * gcp_batch_workspace_size).  A stream's share of a batched call has a work
 * plan of its own (pair blocks per stream; default 1024, fewer and larger
 * blocks than a single stream's since the other streams supply the
 * parallelism).  This call builds one batch over the registered io for
 * each candidate plan (512, 1024, 2048, 4096 blocks per stream), each on a
 * scratch workspace it allocates and frees, times nine single
 * objective+gradient calls per candidate taken round-robin over the
 * candidates, and gives every stream the plan with the lowest median call;
 * or it reads the plan from cache_path, keyed on
 * the device and the batch's shape buckets (see gcp_autotune), and appends
 * a tuned plan there.  The registered outputs are written.  *buckets (may
 * be NULL) receives the number of distinct shape buckets.  Synchronous.
 * Errors: GCP_E_ARG (NULL arguments, n < 1), GCP_E_DEVICE (device calls,
 * including the scratch allocation), or those of gcp_batch_create. */
gcp_status gcp_batch_autotune(gcp_stream* const* streams, const gcp_batch_io* io, int32_t n,
                              const char* cache_path, int32_t* buckets);

gcp_status gcp_batch_workspace_size(gcp_stream* const* streams, int32_t n, size_t* bytes);

/* Builds the batch (synchronous: uploads descriptors and state).  Each
 * gradient call runs one persistent launch per tile build present (loss,
 * rank tile, h-tiles, copy width) over that build's work items; the launches
 * go to up to four HIP streams (hip_stream and three the batch creates and
 * destroys), forked from and joined back into hip_stream with events, so a
 * graph captured on hip_stream holds them as parallel branches. */
gcp_status gcp_batch_create(gcp_stream* const* streams, const gcp_batch_io* io, int32_t n, void* workspace,
                            size_t ws_bytes, hipStream_t hip_stream, gcp_batch** out);

/* Objective and gradients of every stream at its current factors over its
 * registered X_t and window: one persistent launch per tile build present
 * (spread over the batch's HIP streams) plus one reduce launch.
 * Writes the registered outputs (want: GCP_WANT_LOSS | GCP_WANT_GRAD). */
gcp_status gcp_batch_loss_grad(gcp_batch* b, uint32_t want);

/* gcp_update_factors for every stream with its registered X_t and s_t
 * (tau_f and kappa_f of the first stream; all streams must share them):
 * kappa_f = 0: tau_f x [batched gradient, batched ADAM step];
 * kappa_f > 0: Alg. 4's epochs as in gcp_update_factors, per stream on the
 * device (objective with s_t fixed, then per epoch tau_f x [gradient, ADAM
 * step with the stream's device-held rate] and the keep-or-undo decision
 * with Alg. 2's Update: rate x 0.1 and the iteration index back tau_f on an
 * undo; a stream whose objective is at or below tol_f stops stepping);
 * then A_old <- A and the reservoir window update with the draw made on the
 * device, then t <- t+1.  gcp_factor_info reports each stream's solver
 * state after gcp_batch_sync_streams. */
gcp_status gcp_batch_update_factors(gcp_batch* b);

/* Temporal weights (as gcp_solve_st) for every stream of the batch whose
 * solver applies: GCP_TSOLVE_SGD streams and Gaussian-loss GCP_TSOLVE_LS
 * streams, from the registered X_t and current factors, written into the
 * registered s_t buffer (which is then an input/output buffer).  LS streams
 * with other losses keep the s_t their caller wrote.  All launches go to the
 * batch's HIP stream with no host synchronisation; capturable.  A failed
 * Cholesky pivot or a non-finite value is reported by gcp_batch_sync_streams. */
gcp_status gcp_batch_solve_st(gcp_batch* b);

/* One time step of Alg. 1 for every stream: gcp_batch_solve_st, then
 * gcp_batch_update_factors. */
gcp_status gcp_batch_step(gcp_batch* b);

/* Copies the device-side step state back into the stream handles (waits). */
gcp_status gcp_batch_sync_streams(gcp_batch* b);

gcp_status gcp_batch_destroy(gcp_batch* b);

/* The draws that the sampled gradient (Section 4.3, Algorithm 6) forms for
 * one slice at sampler call number `call`: slice h_index (0: X_t, whose
 * membership table is built here; h >= 1: window slot h-1 of a stored-slice
 * stream).  Writes n = p + q draws in draw order (the p nonzero draws, then
 * the q zero draws) into the device buffers coords (n x 3 int32, the
 * multi-index) and weights (n floats: eta/p, zeta/q, or 0 for a zero draw
 * that found no free cell in 64 attempts, which also sets the numeric
 * status); *n (host) = p + q.  COO streams only; cap < p + q gives GCP_E_ARG.
 * The stream's call counter does not advance.  For checking the sampler
 * against its definition: the gradient kernels form their draws with the
 * same device code. */
gcp_status gcp_dump_samples(gcp_stream* s, const gcp_slice* X_t, int32_t h_index, int64_t call,
                            int32_t* coords, float* weights, int64_t cap, int64_t* n);

/* Measurement tooling.  With enable != 0, each following gcp_loss_grad
 * records a pair of HIP events on the stream's HIP stream immediately before
 * and after its main gradient kernel (up to `capacity` pairs; the events are
 * created here, outside any timed region).  gcp_kernel_time waits for the
 * recorded events, returns the summed kernel milliseconds and the number of
 * launches timed, and starts a new count.  enable = 0 destroys the events. */
gcp_status gcp_kernel_timing(gcp_stream* s, int32_t enable, int32_t capacity);
gcp_status gcp_kernel_time(gcp_stream* s, double* total_ms, int64_t* count);

const char* gcp_status_string(gcp_status st);

#ifdef __cplusplus
}
#endif

#endif /* GCPSTREAM_H */
