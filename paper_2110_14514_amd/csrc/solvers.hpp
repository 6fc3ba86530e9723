// Interfaces of the SGD solvers (Algorithms 3 and 4) between the C-ABI shell
// and their kernels.
#pragma once

#include "common.hpp"

namespace gcp {

// Temporal-weight solver of Algorithm 3 on a dense slice (ADAM epochs with
// roll-back, decided on the device).  The workspace of tsgd_ws_bytes bytes
// starts with the solver state.
struct TsgdState {
  double F;          // objective at the last accepted weights
  double alpha;      // current ADAM rate
  int64_t i;         // ADAM iteration index
  double p1, p2;     // beta1^i, beta2^i
  uint64_t rolled;   // bit e set: epoch e was rolled back
  int32_t done;      // stopping test met: later passes do nothing
  int32_t epoch;     // epochs run
  int32_t pad;
};
struct TsgdCall {
  int I1, I2, I3, R, loss, dtype;
  const void* X;
  const void* A[3];
  void* s;           // weights: written from zero, the solver's iterate
  double mu, lower, alpha, beta1, beta2, eps, tol;
  int tau, kappa;
  void* ws;
  int* status;
  hipStream_t stream;
};
size_t tsgd_ws_bytes(int I1, int I2, int I3, int R, int dtype);
hipError_t tsgd_run(const TsgdCall& c);
// Pieces of Algorithm 3 for sampled (COO) slices, whose gradients and
// objective estimates come from the sampled kernels: reset the solver, the
// ADAM Step from a weight gradient g (mu s included), and the start (init)
// or end-of-epoch decision on an estimate *F (mu/2 ||s||^2 included).
hipError_t tsgd_sampled_begin(const TsgdCall& c);
hipError_t tsgd_sampled_step(const TsgdCall& c, const void* g);
hipError_t tsgd_sampled_decide(const TsgdCall& c, const void* F, int init);

// Epochs of the factor solver (Algorithm 4): state kept for the whole stream.
struct FacState {
  double F;          // objective at the last accepted factors
  double alpha;      // current ADAM rate
  double alpha_t;    // bias-corrected rate of the step being taken
  int64_t i;         // ADAM iteration index
  double p1, p2;     // beta1^i, beta2^i
  uint64_t rolled;   // bit e set: epoch e of the last call was rolled back
  int32_t done;      // stopping test met: later steps of the call do nothing
  int32_t epoch;     // epochs run in the last call
  int32_t roll;      // last decision: 1 undo, 0 keep, -1 none
  int32_t pad;
};
hipError_t fac_init_run(FacState* st, double alpha, hipStream_t stream);
// i <- i + 1 and the ADAM Step with the device-held rate (skipped once done).
hipError_t fac_step_run(int dtype, int64_t n, void* a, const void* g, void* u, void* v, FacState* st, double beta1,
                        double beta2, double eps, double lower, hipStream_t stream);
hipError_t fac_begin_run(int dtype, FacState* st, const void* loss, double tol, hipStream_t stream);
// Decision on *loss, then the copy it asks for (n factor entries).
hipError_t fac_end_epoch_run(int dtype, int64_t n, void* a, void* u, void* v, void* ao, void* uo, void* vo,
                             FacState* st, const void* loss, int tau, double tol, double beta1, double beta2,
                             hipStream_t stream);

// Evaluation metrics (Section 6): workspace of metrics_ws_bytes bytes.
size_t metrics_ws_bytes();
// *out (device FP64) = sum of squares of n values of X.
hipError_t sumsq_run(int dtype, const void* X, int64_t n, void* ws, double* out, hipStream_t stream);
// Four-way slices through merged modes 3 and 4 (row i3 I4 + i4):
// out = the merged factor, rows A3[i3] * A4[i4];
hipError_t kr_merge_run(int dtype, const void* A3, const void* A4, int I3, int I4, int R, void* out,
                        hipStream_t stream);
// G3, G4 from the merged mode's gradient G34, plus grad_scale x lam A3/A4;
hipError_t merged_project_run(int dtype, const void* G34, const void* A3, const void* A4, int I3, int I4, int R,
                              double lam, const void* gscale, void* G3, void* G4, int* status, hipStream_t stream);
// *loss += lam/2 (||A3||^2 + ||A4||^2) (n3, n4: entries of A3, A4).
hipError_t merged_reg_run(int dtype, void* loss, const void* A3, int64_t n3, const void* A4, int64_t n4, double lam,
                          hipStream_t stream);
// A bit-packed binary slice (rows of ceil(I3/32) words, entry i3 = bit i3 % 32
// of word i3 / 32) written out as FP32 0/1 values, rows x I3.
hipError_t unpack_bits_run(const void* words, float* out, int64_t rows, int I3, hipStream_t stream);
// Column norms and cross products of two K-tensors' factors (Ra, Rb <= 64),
// laid out at cross_results(ws) as C[3][Ra][Rb], Na[3][Ra], Nb[3][Rb].
hipError_t cross_run(int dtype, const void* const* A, const void* const* B, const int* I, int Ra, int Rb, void* ws,
                     hipStream_t stream);
const double* cross_results(const void* ws);
// p[0..n) = v (at most 256-thread single-workgroup fill; small n).
hipError_t fill_run(int dtype, void* p, int n, double v, hipStream_t stream);
// kMaxRank values inside the metrics workspace reserved for a row of ones.
void* metrics_ones(void* ws);
// *p += v on the device (p: one value of the stream dtype).
hipError_t scalar_add_run(int dtype, void* p, double v, hipStream_t stream);

}  // namespace gcp
