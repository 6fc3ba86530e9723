// C-ABI shell of gcpstream: argument validation, workspace layout, the
// stream's host-side state (time index, window slots, ADAM iteration) and the
// launch sequences of each call.  Declarations and contracts are in
// include/gcpstream.h.
#include "../../include/gcpstream.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <utility>
#include <vector>
#include <mutex>
#include <string>
#include <limits>

#include "solvers.hpp"

using namespace gcp;

struct WsLayout {
  size_t status, A, Aold, u, v, G, gs, loss, shist, ring, part, ls, plain, tab, sorted, hist, tsgd, fac, Ao, uo, vo,
      metric, ident, xf, A34, G34, B34, stamps, total;
  size_t sorted_bytes;    // COO: row-sorted reduction workspace (0: float atomics)
  size_t coo_slot;        // bytes of one COO window slot (coords then values)
  size_t fac_elems;       // sum_k I_k R
  size_t fac_off[4];      // element offsets of A^(k) inside a packed factor block
  size_t plain_bytes, part_bytes;
  uint64_t tab_cap;       // COO: capacity of each membership table (0: dense)
  size_t rp3;             // dense: row pitch of stored slices (I3 rounded up to 32 values;
                          // bit-packed: ceil(I3/32) words)
  size_t slot_elems;      // dense: elements (bit-packed: words) of one stored slice (I1 I2 rp3)
};

struct gcp_stream {
  gcp_params p;
  size_t es;
  size_t omega;
  int dims[3];          // the kernels' slice shape (d = 4: I1, I2, I3 I4)
  int d4[2];            // d = 4: I3 and I4 (modes 3 and 4 merged in the kernels)
  hipStream_t st;
  char* ws;
  WsLayout L;
  int64_t t;
  int nwin;
  std::vector<int64_t> slot_t;     // time stamp of each window slot (host copy)
  int64_t adam_i;
  std::vector<int64_t> slot_nnz;
  int64_t sample_call;
  int* status;
  std::vector<hipEvent_t> ev;   // begin/end pairs for gcp_kernel_timing
  int ev_used;
  int plan_target;              // matrix-core work plan chosen by gcp_autotune (0: automatic)
  int batch_plan_target;        // the plan of the stream's share of a batched call
};

namespace {

// COO streams whose SGD solvers judge epochs by Algorithm 5's estimates.
bool needs_estimates(const gcp_params* p) {
  return p->slice_kind == GCP_SLICE_COO && (p->kappa_f > 0 || p->tsolve == GCP_TSOLVE_SGD);
}

// Call numbers of the estimates of time step t: fixed for a solve, one per
// solver, apart from the gradients' counter (which counts up from 0).
uint32_t factor_estimate_call(int64_t t) { return 0x80000000u | (uint32_t)(t & 0x3FFFFFFF); }
uint32_t weight_estimate_call(int64_t t) { return 0xC0000000u | (uint32_t)(t & 0x3FFFFFFF); }

gcp_status check_params(const gcp_params* p) {
  if (!p) return GCP_E_ARG;
  if (p->abi_version != GCP_ABI_VERSION) return GCP_E_ARG;
  if (p->d != 2 && p->d != 3 && p->d != 4) return GCP_E_UNSUPPORTED;
  if (p->d == 2 && p->dims[2] != 1) return GCP_E_SHAPE;   // matrix slices: dims (I1, I2, 1)
  if (p->d == 2 && p->lower > 1.0) return GCP_E_ARG;       // the fixed row of ones must satisfy the bound
  for (int k = 0; k < (p->d == 4 ? 4 : 3); ++k)
    if (p->dims[k] < 1 || p->dims[k] > (1 << 30)) return GCP_E_SHAPE;
  if (p->d == 4) {
    // four-way slices: modes 3 and 4 merged in the kernels
    if ((double)p->dims[2] * p->dims[3] > (double)(1 << 30)) return GCP_E_SHAPE;
    if (p->slice_kind != GCP_SLICE_DENSE || p->hist != GCP_HIST_SLICES) return GCP_E_UNSUPPORTED;
    if (p->flags & (GCP_FLAG_GAUSS_IDENTITY | GCP_FLAG_PLAIN_SCRATCH)) return GCP_E_UNSUPPORTED;
  }
  if ((double)p->dims[0] * p->dims[1] * p->dims[2] * (p->d == 4 ? p->dims[3] : 1) > 9.0e15) return GCP_E_SHAPE;
  if ((double)p->dims[0] * p->dims[1] >= 2147483647.0) return GCP_E_SHAPE;
  if (p->rank < 1 || p->rank > GCP_MAX_RANK) return GCP_E_ARG;
  if (p->window < 0 || p->window > (p->hist == GCP_HIST_MODEL ? GCP_MAX_WINDOW_MODEL : GCP_MAX_WINDOW))
    return GCP_E_ARG;
  if (p->loss < 0 || p->loss > 4) return GCP_E_ARG;
  if (p->dtype != GCP_F32 && p->dtype != GCP_F64) return GCP_E_ARG;
  if (p->slice_kind != GCP_SLICE_DENSE && p->slice_kind != GCP_SLICE_COO && p->slice_kind != GCP_SLICE_BITS)
    return GCP_E_UNSUPPORTED;
  if (p->slice_kind == GCP_SLICE_BITS) {
    // bit-packed binary slices: read by the matrix-core kernels only
    if (p->loss != GCP_LOSS_BERNOULLI_LOGIT && p->loss != GCP_LOSS_BERNOULLI_ODDS) return GCP_E_UNSUPPORTED;
    if (p->dtype != GCP_F32 || p->d != 3 || p->window > 31 || p->rank > 32) return GCP_E_UNSUPPORTED;
    if (p->hist != GCP_HIST_SLICES) return GCP_E_UNSUPPORTED;
    if (p->flags & (GCP_FLAG_KERNEL_VALU | GCP_FLAG_PLAIN_SCRATCH)) return GCP_E_UNSUPPORTED;
  }
  if (p->slice_kind == GCP_SLICE_COO) {
    if (p->dtype != GCP_F32) return GCP_E_UNSUPPORTED;
    if (p->p < 0 || p->q < 0 || p->p + p->q < 1) return GCP_E_ARG;
    if (p->max_nnz < 1 || p->max_nnz >= ((int64_t)1 << 32)) return GCP_E_ARG;
    if (p->flags & GCP_FLAG_PLAIN_SCRATCH) return GCP_E_UNSUPPORTED;
    if (p->dims[0] * p->dims[1] * p->dims[2] >= ((int64_t)1 << 62)) return GCP_E_SHAPE;
  }
  if (!(p->theta > 0.0 && p->theta <= 1.0)) return GCP_E_ARG;
  if (!isfinite(p->w) || !isfinite(p->lambda) || !isfinite(p->mu) || p->lambda < 0 || p->mu < 0)
    return GCP_E_ARG;
  if (isnan(p->lower) || p->lower == INFINITY) return GCP_E_ARG;
  if (p->tau_f < 0) return GCP_E_ARG;
  if (!(p->beta1 >= 0 && p->beta1 < 1 && p->beta2 >= 0 && p->beta2 < 1 && p->adam_eps > 0))
    return GCP_E_ARG;
  if ((p->flags & GCP_FLAG_PLAIN_SCRATCH) && p->dtype != GCP_F32) return GCP_E_UNSUPPORTED;
  if ((p->flags & GCP_FLAG_KERNEL_VALU) && (p->flags & GCP_FLAG_KERNEL_MFMA)) return GCP_E_ARG;
  if (p->flags & ~(GCP_FLAG_PLAIN_SCRATCH | GCP_FLAG_KERNEL_VALU | GCP_FLAG_KERNEL_MFMA | GCP_FLAG_SAMPLED_ATOMIC |
                   GCP_FLAG_GAUSS_IDENTITY))
    return GCP_E_ARG;
  if ((p->flags & GCP_FLAG_GAUSS_IDENTITY) && (p->loss != GCP_LOSS_GAUSSIAN || p->slice_kind != GCP_SLICE_DENSE))
    return GCP_E_ARG;
  if ((p->flags & GCP_FLAG_SAMPLED_ATOMIC) && p->slice_kind != GCP_SLICE_COO) return GCP_E_ARG;
  if (p->hist != GCP_HIST_SLICES && p->hist != GCP_HIST_MODEL) return GCP_E_ARG;
  if (p->kappa_f < 0 || p->kappa_f > 64 || isnan(p->tol_f)) return GCP_E_ARG;
  if (needs_estimates(p) && (p->p_est < 0 || p->q_est < 0 || p->p_est + p->q_est < 1)) return GCP_E_ARG;
  if (p->tsolve != GCP_TSOLVE_LS && p->tsolve != GCP_TSOLVE_SGD) return GCP_E_ARG;
  if (p->tsolve == GCP_TSOLVE_SGD) {
    if (p->tau_w < 1 || p->kappa_w < 0 || p->kappa_w > 64) return GCP_E_ARG;
    if (!(p->alpha_w > 0.0) || !isfinite(p->alpha_w) || isnan(p->tol_w)) return GCP_E_ARG;
  }
  return GCP_OK;
}

WsLayout layout_for(const gcp_params* p) {
  WsLayout L;
  const size_t es = p->dtype == GCP_F64 ? 8 : 4;
  // d = 4: the slice geometry is I1 x I2 x (I3 I4); the factor blocks keep
  // the four modes
  const bool four = p->d == 4;
  const int I1 = (int)p->dims[0], I2 = (int)p->dims[1], R = p->rank;
  const int I3 = four ? (int)(p->dims[2] * p->dims[3]) : (int)p->dims[2];
  const size_t omega = (size_t)I1 * I2 * I3;
  L.fac_off[0] = 0;
  L.fac_off[1] = (size_t)I1 * R;
  L.fac_off[2] = L.fac_off[1] + (size_t)I2 * R;
  L.fac_off[3] = L.fac_off[2] + (size_t)p->dims[2] * R;
  L.fac_elems = four ? L.fac_off[3] + (size_t)p->dims[3] * R : L.fac_off[2] + (size_t)I3 * R;
  const size_t fb = align_up(L.fac_elems * es, 256);
  size_t off = 0;
  L.status = off; off += 256;
  L.A = off; off += fb;
  L.Aold = off; off += fb;
  L.u = off; off += fb;
  L.v = off; off += fb;
  L.G = off; off += fb;
  L.gs = off; off = align_up(off + (size_t)R * es, 256);
  L.loss = off; off += 256;
  L.shist = off; off = align_up(off + (size_t)p->window * R * es, 256);
  const bool coo = p->slice_kind == GCP_SLICE_COO;
  const bool model = p->hist == GCP_HIST_MODEL;
  // slices kept in the window (the model-difference history keeps none)
  const int wslices = model ? 0 : p->window;
  L.coo_slot = coo ? align_up((size_t)p->max_nnz * 16, 256) : 0;
  // stored dense slices keep each (i1, i2) row on 128-byte lines: the row
  // pitch is I3 rounded up to 32 values (the padding is zeroed at set-up
  // and read only as the zero tail of a 16-byte copy);
  // bit-packed slices keep their own layout, ceil(I3/32) words per row
  const bool bits = p->slice_kind == GCP_SLICE_BITS;
  L.rp3 = bits ? ((size_t)I3 + 31) / 32 : ((size_t)I3 + 31) / 32 * 32;
  L.slot_elems = (size_t)I1 * I2 * L.rp3;
  L.ring = off;
  off = align_up(off + (coo ? (size_t)wslices * L.coo_slot : (size_t)wslices * L.slot_elems * es), 256);
  L.part_bytes = coo ? 0 : dense_fused_part_bytes(I1, I2, I3, R, p->dtype);
  L.part = off; off = align_up(off + L.part_bytes, 256);
  L.ls = off; off = align_up(off + (coo ? 0 : ls_scratch_bytes(I1, I2, I3, R)), 256);
  L.plain_bytes = (p->flags & GCP_FLAG_PLAIN_SCRATCH) ? dense_plain_scratch_bytes(I1, I2, I3, R, p->dtype) : 0;
  L.plain = off; off = align_up(off + L.plain_bytes, 256);
  // COO: one membership table per window slot and one for the current slice
  L.tab_cap = coo ? table_capacity(p->max_nnz) : 0;
  L.tab = off; off = align_up(off + (size_t)(coo ? wslices + 1 : 0) * L.tab_cap * 8, 256);
  L.sorted_bytes = (coo && !(p->flags & GCP_FLAG_SAMPLED_ATOMIC))
                       ? sampled_sorted_bytes(I1, I2, I3, R, wslices, p->p, p->q)
                       : 0;
  L.sorted = off; off = align_up(off + L.sorted_bytes, 256);
  L.hist = off; off = align_up(off + (model ? hist_ws_bytes(R) : 0), 256);
  L.tsgd = off;
  off = align_up(off + (p->tsolve == GCP_TSOLVE_SGD ? tsgd_ws_bytes(I1, I2, I3, R, p->dtype == GCP_F64) : 0), 256);
  // factor epochs: state, objective scalar, saved factors and moments
  const bool epochs = p->kappa_f > 0;
  L.fac = off; off += epochs ? 512 : 0;
  L.Ao = off; off += epochs ? fb : 0;
  L.uo = off; off += epochs ? fb : 0;
  L.vo = off; off += epochs ? fb : 0;
  L.metric = off; off += align_up(metrics_ws_bytes(), 256);
  L.ident = off; off = align_up(off + ((p->flags & GCP_FLAG_GAUSS_IDENTITY) ? hist_ws_bytes(R) : 0), 256);
  // bit-packed streams: one slice as FP32 values for the solvers and
  // metrics that read floats (the weights' SGD solve, slice losses)
  L.xf = off; off = align_up(off + (bits ? omega * 4 : 0), 256);
  // d = 4: the merged mode's factor rows (the stream's, and a reference
  // K-tensor's for the score) and its gradient
  const size_t m34 = four ? (size_t)I3 * R * es : 0;
  L.A34 = off; off = align_up(off + m34, 256);
  L.G34 = off; off = align_up(off + m34, 256);
  L.B34 = off; off = align_up(off + m34, 256);
  // the window's slot time stamps on the device (the history kernels form
  // w_h from them; up to GCP_MAX_WINDOW_MODEL slots)
  L.stamps = off; off = align_up(off + (size_t)std::max(1, p->window) * 8, 256);
  L.total = off;
  return L;
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

bool bits_stream(const gcp_stream* s) { return s->p.slice_kind == GCP_SLICE_BITS; }

// Dense slices (FP values, 16-byte aligned) or bit-packed ones (words,
// 4-byte aligned), whichever the stream holds.
gcp_status check_dense_slice(const gcp_stream* s, const gcp_slice* X) {
  if (!X || !X->vals) return GCP_E_ARG;
  if (s->p.slice_kind == GCP_SLICE_BITS) {
    if (X->kind != GCP_SLICE_BITS) return GCP_E_ARG;
    if ((uintptr_t)X->vals & 3u) return GCP_E_ALIGN;
    return GCP_OK;
  }
  if (X->kind != GCP_SLICE_DENSE || s->p.slice_kind != GCP_SLICE_DENSE) return GCP_E_ARG;
  if (!aligned16(X->vals)) return GCP_E_ALIGN;
  return GCP_OK;
}

gcp_status check_coo_slice(const gcp_stream* s, const gcp_slice* X) {
  if (!X || X->kind != GCP_SLICE_COO || s->p.slice_kind != GCP_SLICE_COO) return GCP_E_ARG;
  if (X->nnz < 0 || X->nnz > s->p.max_nnz) return GCP_E_SHAPE;   // tables hold max_nnz entries
  if (X->nnz > 0 && (!X->vals || !X->coords)) return GCP_E_ARG;
  if (s->p.p > 0 && X->nnz == 0) return GCP_E_ARG;               // no nonzero to draw
  if (s->p.q > 0 && (int64_t)s->omega - X->nnz <= 0) return GCP_E_ARG;  // no zero to draw
  if (needs_estimates(&s->p) && s->p.p_est > 0 && X->nnz == 0) return GCP_E_ARG;
  if (needs_estimates(&s->p) && s->p.q_est > 0 && (int64_t)s->omega - X->nnz <= 0) return GCP_E_ARG;
  if (((uintptr_t)X->coords & 3u) || ((uintptr_t)X->vals & 3u)) return GCP_E_ALIGN;
  return GCP_OK;
}

char* coo_slot_coords(gcp_stream* s, int slot) { return s->ws + s->L.ring + (size_t)slot * s->L.coo_slot; }
char* coo_slot_vals(gcp_stream* s, int slot) {
  return coo_slot_coords(s, slot) + (size_t)s->p.max_nnz * 12;
}

// Copy a dense slice (row pitch I3) into window slot `slot` (row pitch rp3);
// a bit-packed slice has the slot's layout already.
hipError_t store_dense_slot(gcp_stream* s, int slot, const void* vals) {
  if (s->p.slice_kind == GCP_SLICE_BITS)
    return hipMemcpyAsync(s->ws + s->L.ring + (size_t)slot * s->L.slot_elems * 4, vals, s->L.slot_elems * 4,
                          hipMemcpyDeviceToDevice, s->st);
  const size_t w = (size_t)s->dims[2] * s->es;
  return hipMemcpy2DAsync(s->ws + s->L.ring + (size_t)slot * s->L.slot_elems * s->es, s->L.rp3 * s->es, vals, w, w,
                          (size_t)s->dims[0] * s->dims[1], hipMemcpyDeviceToDevice, s->st);
}

// Membership table of window slot `slot`; slot == window: the current slice's.
uint64_t* coo_table(gcp_stream* s, int slot) {
  return reinterpret_cast<uint64_t*>(s->ws + s->L.tab + (size_t)slot * s->L.tab_cap * 8);
}

bool model_hist(const gcp_stream* s) { return s->p.hist == GCP_HIST_MODEL; }

// Window slices kept by the stream (the model-difference history keeps none).
int window_slices(const gcp_stream* s) { return model_hist(s) ? 0 : s->p.window; }

// Membership table of the current slice: after those of the window slots.
uint64_t* current_table(gcp_stream* s) { return coo_table(s, window_slices(s)); }

hipError_t store_coo_slot(gcp_stream* s, int slot, const gcp_slice* X) {
  hipError_t e = hipSuccess;
  if (X->nnz > 0) {
    e = hipMemcpyAsync(coo_slot_coords(s, slot), X->coords, (size_t)X->nnz * 12, hipMemcpyDeviceToDevice, s->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(coo_slot_vals(s, slot), X->vals, (size_t)X->nnz * 4, hipMemcpyDeviceToDevice, s->st);
  }
  if (e == hipSuccess)
    e = table_build(reinterpret_cast<const int32_t*>(coo_slot_coords(s, slot)), X->nnz, s->dims[1], s->dims[2],
                    coo_table(s, slot), s->L.tab_cap, s->st);
  s->slot_nnz[slot] = X->nnz;
  return e;
}

// Table of the current slice X_t, rebuilt for every call that samples it.
hipError_t build_current_table(gcp_stream* s, const gcp_slice* X_t) {
  return table_build(X_t->coords, X_t->nnz, s->dims[1], s->dims[2], current_table(s), s->L.tab_cap, s->st);
}

SampledCall sampled_call(gcp_stream* s, const gcp_slice* X_t, const void* const* A, const void* s_t, int want,
                         void* loss, void* const* G, void* g_s, int64_t call = -1) {
  SampledCall c;
  memset(&c, 0, sizeof(c));
  c.I1 = s->dims[0]; c.I2 = s->dims[1]; c.I3 = s->dims[2]; c.R = s->p.rank;
  c.loss = s->p.loss; c.want = want;
  c.coords[0] = X_t->coords; c.vals[0] = X_t->vals; c.nnz[0] = X_t->nnz; c.stamp[0] = s->t;
  c.tab[0] = current_table(s);
  c.tab_cap = s->L.tab_cap;
  c.S[0] = s_t; c.c[0] = 1.0;
  int n = 1;
  for (int slot = 0; slot < (model_hist(s) ? 0 : s->nwin); ++slot, ++n) {
    c.coords[n] = reinterpret_cast<const int32_t*>(coo_slot_coords(s, slot));
    c.tab[n] = coo_table(s, slot);
    c.vals[n] = coo_slot_vals(s, slot);
    c.nnz[n] = s->slot_nnz[slot];
    c.stamp[n] = s->slot_t[slot];
    c.S[n] = s->ws + s->L.shist + (size_t)slot * s->p.rank * s->es;
    c.c[n] = s->p.w * pow(s->p.theta, (double)(s->t - s->slot_t[slot]));
  }
  c.ns = n;
  for (int k = 0; k < 3; ++k) {
    c.A[k] = A[k];
    c.G[k] = G[k];
  }
  c.gs = g_s; c.loss_out = loss;
  c.lam = s->p.lambda; c.mu = s->p.mu;
  c.p = s->p.p; c.q = s->p.q; c.seed = s->p.seed;
  // a sampled evaluation takes the next call number; a sample dump names its own
  c.call = call >= 0 ? call : s->sample_call++;
  c.status = s->status; c.stream = s->st;
  if (s->L.sorted_bytes) sampled_sorted_bind(c, s->ws + s->L.sorted, window_slices(s));
  return c;
}

char* fac_ptr(gcp_stream* s, size_t block, int k) { return s->ws + block + s->L.fac_off[k] * s->es; }

bool four_way(const gcp_stream* s) { return s->p.d == 4; }

// The kernels' three factors for the caller's factors A (k < d): with d = 4
// the third is the merged modes 3 and 4, formed into the workspace at
// `scratch` (rows A3[i3] * A4[i4], rank R).
hipError_t kernel_factors(gcp_stream* s, const void* const* A, const void* out[3], size_t scratch, int R) {
  out[0] = A[0];
  out[1] = A[1];
  if (!four_way(s)) {
    out[2] = A[2];
    return hipSuccess;
  }
  void* dst = s->ws + scratch;
  out[2] = dst;
  return kr_merge_run(s->p.dtype == GCP_F64, A[2], A[3], s->d4[0], s->d4[1], R, dst, s->st);
}

// After a kernel call on merged modes: G3 and G4 from the merged gradient
// (L.G34), and the objective's regulariser on A3 and A4 (the kernels put
// none on the merged mode).  lam: the call's regulariser weight.
hipError_t finish_four_way(gcp_stream* s, const void* const* A, int want, double lam, void* loss, void* G3, void* G4,
                           const void* grad_scale) {
  if (!four_way(s)) return hipSuccess;
  const int dt = s->p.dtype == GCP_F64;
  const int I3 = s->d4[0], I4 = s->d4[1], R = s->p.rank;
  hipError_t e = hipSuccess;
  if (want & kWantGrad)
    e = merged_project_run(dt, s->ws + s->L.G34, A[2], A[3], I3, I4, R, lam, grad_scale, G3, G4, s->status, s->st);
  if (e == hipSuccess && (want & kWantLoss) && loss && lam != 0.0)
    e = merged_reg_run(dt, loss, A[2], (int64_t)I3 * R, A[3], (int64_t)I4 * R, lam, s->st);
  return e;
}

void fill_window(gcp_stream* s, DenseCall& c) {
  c.ring = s->ws + s->L.ring;
  c.ring_pitch = s->L.rp3;
  c.ring_stride = s->L.slot_elems;
  c.shist = s->ws + s->L.shist;
  c.omega = s->omega;
  int n = 1;
  for (int slot = 0; slot < (model_hist(s) ? 0 : s->nwin); ++slot, ++n) {
    c.X[n] = s->ws + s->L.ring + (size_t)slot * s->L.slot_elems * s->es;
    c.S[n] = s->ws + s->L.shist + (size_t)slot * s->p.rank * s->es;
    c.c[n] = s->p.w * pow(s->p.theta, (double)(s->t - s->slot_t[slot]));
  }
  c.ns = n;
}

DenseCall base_call(gcp_stream* s) {
  DenseCall c;
  memset(&c, 0, sizeof(c));
  c.I1 = s->dims[0];
  c.I2 = s->dims[1];
  c.I3 = s->dims[2];
  c.R = s->p.rank;
  c.loss = s->p.loss;
  c.dtype = s->p.dtype;
  c.lam = s->p.lambda;
  c.mu = s->p.mu;
  c.part = s->ws + s->L.part;
  c.part_bytes = s->L.part_bytes;
  c.status = s->status;
  c.stream = s->st;
  c.c[0] = 1.0;
  c.kernel = (s->p.flags & GCP_FLAG_KERNEL_VALU) ? 1 : ((s->p.flags & GCP_FLAG_KERNEL_MFMA) ? 2 : 0);
  c.plan_target = s->plan_target;
  c.xbits = s->p.slice_kind == GCP_SLICE_BITS;
  return c;
}

gcp_status hip_status(hipError_t e) { return e == hipSuccess ? GCP_OK : GCP_E_DEVICE; }

// Factor entries that take ADAM steps: every block of the packed layout.  For
// matrix slices the fixed row of ones (the middle block) is included; it
// stays put because its gradient is cleared before every step and adam_eps
// is required to be positive (a zero gradient then gives a zero step).
int64_t adam_elems(const gcp_stream* s) { return (int64_t)s->L.fac_elems; }

// Matrix slices are carried as I1 x 1 x I2 tensors (the same memory as the
// I1 x I2 row-major slice, so that i2 runs along the lanes): the caller's
// modes 0 and 1 are internal modes 0 and 2, and internal mode 1 is a fixed
// 1 x R row of ones.  Internal mode of the caller's mode k:
int int_mode(const gcp_stream* s, int k) { return s->p.d == 2 && k == 1 ? 2 : (s->p.d == 2 && k == 2 ? 1 : k); }

// The parameters as the stream keeps them (matrix slices: dims (I1, 1, I2)).
gcp_params internal_params(const gcp_params* p) {
  gcp_params q = *p;
  if (p->d == 2) {
    q.dims[2] = p->dims[1];
    q.dims[1] = 1;
  }
  return q;
}

// The fixed row takes no ADAM steps: its gradient is cleared after each
// gradient (ADAM moves nothing with zero moments and a zero gradient).
hipError_t d2_clear_fixed_grad(gcp_stream* s) {
  if (s->p.d != 2) return hipSuccess;
  return fill_run(s->p.dtype == GCP_F64, fac_ptr(s, s->L.G, 1), s->p.rank, 0.0, s->st);
}

// Gradient-only Gaussian calls of a stream with GCP_FLAG_GAUSS_IDENTITY go
// through the identity of Section 5: a data pass without the model, then the
// model's part from Gram matrices.
bool use_identity(const gcp_stream* s, int want, bool plain, const void* grad_scale) {
  return (s->p.flags & GCP_FLAG_GAUSS_IDENTITY) && want == kWantGrad && !plain && !grad_scale;
}

hipError_t identity_terms(gcp_stream* s, const DenseCall& c) {
  HistCall h;
  memset(&h, 0, sizeof(h));
  for (int k = 0; k < 3; ++k) {
    h.I[k] = s->dims[k];
    h.A[k] = c.A[k];
    h.G[k] = c.G[k];
  }
  h.R = s->p.rank;
  h.dtype = s->p.dtype == GCP_F64 ? 1 : 0;
  h.nwin = c.ns - 1;
  h.stamps = reinterpret_cast<const int64_t*>(s->ws + s->L.stamps);
  h.t = s->t;
  h.w = s->p.w;
  h.theta = s->p.theta;
  h.shist = s->ws + s->L.shist;
  h.ws = reinterpret_cast<double*>(s->ws + s->L.ident);
  h.status = s->status;
  h.stream = s->st;
  return ident_run(h, c.S[0], c.gs);
}

// Matrix slices: the kernels' factor regulariser also covers the fixed row
// (lambda/2 R); take it out of an objective value on the device.
hipError_t d2_fix_loss(gcp_stream* s, void* loss) {
  if (s->p.d != 2 || s->p.lambda == 0.0 || !loss) return hipSuccess;
  return scalar_add_run(s->p.dtype == GCP_F64, loss, -0.5 * s->p.lambda * s->p.rank, s->st);
}

// Algorithm 3 on X (dense, pitch I3) with the stream's factors A, iterating in s_t.
TsgdCall tsgd_call(gcp_stream* s, const void* X, const void* const* A, void* s_t, int* status) {
  TsgdCall c;
  c.I1 = s->dims[0];
  c.I2 = s->dims[1];
  c.I3 = s->dims[2];
  c.R = s->p.rank;
  c.loss = s->p.loss;
  c.dtype = s->p.dtype == GCP_F64;
  c.X = X;
  for (int k = 0; k < 3; ++k) c.A[k] = A[k];
  c.s = s_t;
  c.mu = s->p.mu;
  c.lower = s->p.lower;
  c.alpha = s->p.alpha_w;
  c.beta1 = s->p.beta1;
  c.beta2 = s->p.beta2;
  c.eps = s->p.adam_eps;
  c.tol = s->p.tol_w;
  c.tau = s->p.tau_w;
  c.kappa = s->p.kappa_w;
  c.ws = s->ws + s->L.tsgd;
  c.status = status;
  c.stream = s->st;
  return c;
}

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

void gcp_params_default(gcp_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->abi_version = GCP_ABI_VERSION;
  p->d = 3;
  p->rank = 1;
  p->loss = GCP_LOSS_GAUSSIAN;
  p->dtype = GCP_F32;
  p->slice_kind = GCP_SLICE_DENSE;
  p->w = 1.0;
  p->theta = 1.0;
  p->lambda = 0.0;
  p->mu = 0.0;
  p->lower = -INFINITY;
  p->alpha_f = 1e-3;
  p->beta1 = 0.9;
  p->beta2 = 0.999;
  p->adam_eps = 1e-8;
  p->tau_f = 1;
  p->tsolve = GCP_TSOLVE_LS;
  p->tau_w = 100;
  p->kappa_w = 20;
  p->alpha_w = 1.0;
  p->tol_w = -INFINITY;
  p->kappa_f = 0;
  p->tol_f = -INFINITY;
  p->p_est = 0;
  p->q_est = 0;
}

gcp_status gcp_workspace_size(const gcp_params* p, size_t* bytes) {
  if (!bytes) return GCP_E_ARG;
  gcp_status st = check_params(p);
  if (st != GCP_OK) return st;
  const gcp_params q = internal_params(p);
  *bytes = layout_for(&q).total;
  return GCP_OK;
}

gcp_status gcp_stream_init(const gcp_params* p, const void* const* A0, int32_t n_hist, const gcp_slice* X_hist,
                           const void* s_hist, const int64_t* t_hist, void* workspace, size_t ws_bytes,
                           hipStream_t hip_stream, gcp_stream** out) {
  if (!out) return GCP_E_ARG;
  *out = nullptr;
  gcp_status st = check_params(p);
  if (st != GCP_OK) return st;
  if (!A0 || !A0[0] || !A0[1] || (!A0[2] && p->d >= 3) || (p->d == 4 && !A0[3]) || !workspace) return GCP_E_ARG;
  if (n_hist < 0 || n_hist > p->window) return GCP_E_ARG;
  const bool model = p->hist == GCP_HIST_MODEL;
  if (n_hist > 0 && (!s_hist || !t_hist || (!model && !X_hist))) return GCP_E_ARG;
  if (((uintptr_t)workspace & 255u) != 0) return GCP_E_ALIGN;
  const gcp_params q = internal_params(p);
  WsLayout L = layout_for(&q);
  if (ws_bytes < L.total) return GCP_E_WORKSPACE;
  for (int h = 0; h < n_hist; ++h) {
    if (model) {
      // only the weights and time stamps of the window are kept
    } else if (p->slice_kind == GCP_SLICE_DENSE || p->slice_kind == GCP_SLICE_BITS) {
      if (X_hist[h].kind != p->slice_kind || !X_hist[h].vals) return GCP_E_ARG;
      if (!aligned16(X_hist[h].vals)) return GCP_E_ALIGN;
    } else {
      if (X_hist[h].kind != GCP_SLICE_COO || X_hist[h].nnz < 0 || X_hist[h].nnz > p->max_nnz) return GCP_E_SHAPE;
      if (X_hist[h].nnz > 0 && (!X_hist[h].vals || !X_hist[h].coords)) return GCP_E_ARG;
      if ((p->p > 0 || (needs_estimates(p) && p->p_est > 0)) && X_hist[h].nnz == 0) return GCP_E_ARG;
      if ((p->q > 0 || (needs_estimates(p) && p->q_est > 0)) && X_hist[h].nnz >= p->dims[0] * p->dims[1] * p->dims[2])
        return GCP_E_ARG;
    }
    if (h > 0 && t_hist[h] <= t_hist[h - 1]) return GCP_E_ARG;
    if (t_hist[h] < 1) return GCP_E_ARG;
  }
  gcp_stream* s = new (std::nothrow) gcp_stream();
  if (!s) return GCP_E_ARG;
  s->p = q;
  s->plan_target = 0;
  s->batch_plan_target = kBatchPlanTarget;
  s->es = p->dtype == GCP_F64 ? 8 : 4;
  for (int k = 0; k < 3; ++k) s->dims[k] = (int)q.dims[k];
  s->d4[0] = s->d4[1] = 0;
  if (p->d == 4) {
    s->d4[0] = (int)p->dims[2];
    s->d4[1] = (int)p->dims[3];
    s->dims[2] = (int)(p->dims[2] * p->dims[3]);
  }
  s->omega = (size_t)s->dims[0] * s->dims[1] * s->dims[2];
  s->st = hip_stream;
  s->ws = static_cast<char*>(workspace);
  s->L = L;
  s->status = reinterpret_cast<int*>(s->ws + L.status);
  s->nwin = n_hist;
  s->t = n_hist > 0 ? t_hist[n_hist - 1] + 1 : 1;
  s->slot_t.assign((size_t)std::max(1, p->window), 0);
  s->slot_nnz.assign((size_t)std::max(1, p->window), 0);
  for (int h = 0; h < n_hist; ++h) s->slot_t[h] = t_hist[h];
  hipError_t e = hipMemsetAsync(s->ws + L.status, 0, 256, s->st);
  // matrix slices (d = 2): the third factor is a fixed 1 x R row of ones
  std::vector<double> ones64(p->rank, 1.0);
  std::vector<float> ones32(p->rank, 1.f);
  for (int k = 0; k < (p->d == 4 ? 4 : 3) && e == hipSuccess; ++k) {
    size_t nb = (size_t)q.dims[k] * p->rank * s->es;   // internal shape (d = 2: I1, 1, I2)
    const bool fixed = k == 1 && p->d == 2;
    const void* src = fixed ? (s->es == 8 ? (const void*)ones64.data() : (const void*)ones32.data())
                            : A0[p->d == 2 && k == 2 ? 1 : k];
    const hipMemcpyKind kind = fixed ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    e = hipMemcpyAsync(fac_ptr(s, L.A, k), src, nb, kind, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(fac_ptr(s, L.Aold, k), src, nb, kind, s->st);
  }
  if (e == hipSuccess && p->d == 2)
    e = fill_run(s->es == 8, metrics_ones(s->ws + L.metric), GCP_MAX_RANK, 1.0, s->st);
  if (e == hipSuccess && p->d == 2) e = hipStreamSynchronize(s->st);   // the host row must outlive its copies
  if (e == hipSuccess) e = hipMemsetAsync(s->ws + L.u, 0, L.fac_elems * s->es, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(s->ws + L.v, 0, L.fac_elems * s->es, s->st);
  // the padding of stored rows past I3 must hold finite values: the
  // matrix-core kernels copy rows 16 bytes at a time
  if (e == hipSuccess && p->slice_kind == GCP_SLICE_DENSE && !model && p->window > 0 &&
      s->L.rp3 != (size_t)s->dims[2])
    e = hipMemsetAsync(s->ws + s->L.ring, 0, (size_t)p->window * s->L.slot_elems * s->es, s->st);
  if (e == hipSuccess && p->kappa_f > 0) {
    e = fac_init_run(reinterpret_cast<FacState*>(s->ws + L.fac), p->alpha_f, s->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->ws + L.Ao, s->ws + L.A, L.fac_elems * s->es, hipMemcpyDeviceToDevice, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->ws + L.uo, 0, L.fac_elems * s->es, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->ws + L.vo, 0, L.fac_elems * s->es, s->st);
  }
  for (int h = 0; h < n_hist && e == hipSuccess; ++h) {
    if (model)
      ;
    else if (p->slice_kind == GCP_SLICE_COO)
      e = store_coo_slot(s, h, &X_hist[h]);
    else
      e = store_dense_slot(s, h, X_hist[h].vals);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->ws + L.shist + (size_t)h * p->rank * s->es,
                         static_cast<const char*>(s_hist) + (size_t)h * p->rank * s->es, p->rank * s->es,
                         hipMemcpyDeviceToDevice, s->st);
  }
  // the window's time stamps on the device (the host array is the caller's:
  // wait for the copy)
  if (e == hipSuccess && n_hist > 0) {
    e = hipMemcpyAsync(s->ws + L.stamps, t_hist, (size_t)n_hist * 8, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  }
  if (e != hipSuccess) {
    delete s;
    return GCP_E_DEVICE;
  }
  *out = s;
  return GCP_OK;
}

// The model-difference history term for factors A (previous step's factors:
// the stream's A_old), added to *loss and G after the data term.
static hipError_t add_model_history(gcp_stream* s, const void* const* A, int want, void* loss, void* const* G,
                             const void* grad_scale) {
  if (!model_hist(s) || s->nwin == 0) return hipSuccess;
  HistCall h;
  for (int k = 0; k < 3; ++k) {
    h.I[k] = s->dims[k];
    h.A[k] = A[k];
    h.Ab[k] = fac_ptr(s, s->L.Aold, k);
    h.G[k] = G[k];
  }
  h.R = s->p.rank;
  h.nwin = s->nwin;
  h.dtype = s->p.dtype == GCP_F64 ? 1 : 0;
  h.want = want;
  h.shist = s->ws + s->L.shist;
  h.stamps = reinterpret_cast<const int64_t*>(s->ws + s->L.stamps);
  h.t = s->t;
  h.w = s->p.w;
  h.theta = s->p.theta;
  h.loss = loss;
  h.grad_scale = grad_scale;
  h.ws = reinterpret_cast<double*>(s->ws + s->L.hist);
  h.status = s->status;
  h.stream = s->st;
  return hist_run(h);
}

gcp_status gcp_loss_grad(gcp_stream* s, const gcp_slice* X_t, const void* const* A, const void* s_t, uint32_t want,
                         void* loss, void* const* G, void* g_s) {
  return gcp_loss_grad_scaled(s, X_t, A, s_t, want, nullptr, loss, G, g_s);
}

gcp_status gcp_loss_grad_scaled(gcp_stream* s, const gcp_slice* X_t, const void* const* A_in, const void* s_t,
                                uint32_t want, const void* grad_scale, void* loss, void* const* G_in, void* g_s) {
  if (!s || !A_in || !A_in[0] || !A_in[1] || !s_t) return GCP_E_ARG;
  const bool d2 = s->p.d == 2, d4 = four_way(s);
  if (!A_in[2] && !d2) return GCP_E_ARG;
  if (d4 && !A_in[3]) return GCP_E_ARG;
  if (want & ~(uint32_t)(GCP_WANT_LOSS | GCP_WANT_GRAD | GCP_IMPL_PLAIN)) return GCP_E_ARG;
  if (!(want & (GCP_WANT_LOSS | GCP_WANT_GRAD))) return GCP_E_ARG;
  if ((want & GCP_WANT_LOSS) && !loss) return GCP_E_ARG;
  if ((want & GCP_WANT_GRAD) && d4 && (!G_in || !G_in[2] || !G_in[3])) return GCP_E_ARG;
  // matrix slices: the caller's two factors are internal modes 0 and 2; the
  // fixed row is the stream's own, its gradient goes to scratch.  Four-way
  // slices: the kernels see modes 3 and 4 merged (gradient into scratch,
  // projected afterwards).
  const void* A[3] = {A_in[0], d2 ? fac_ptr(s, s->L.A, 1) : A_in[1], d2 ? A_in[1] : A_in[2]};
  void* Gv[3] = {nullptr, nullptr, nullptr};
  if (G_in) {
    Gv[0] = G_in[0];
    Gv[1] = d2 ? fac_ptr(s, s->L.G, 1) : G_in[1];
    Gv[2] = d2 ? G_in[1] : (d4 ? s->ws + s->L.G34 : G_in[2]);
  }
  void* const* G = G_in ? Gv : nullptr;
  if ((want & GCP_WANT_GRAD) && (!G || !G[0] || !G[1] || !G[2] || !g_s)) return GCP_E_ARG;
  if (d4) {
    hipError_t em = kernel_factors(s, A_in, A, s->L.A34, s->p.rank);
    if (em != hipSuccess) return hip_status(em);
  }
  if (s->p.slice_kind == GCP_SLICE_COO) {
    gcp_status st = check_coo_slice(s, X_t);
    if (st != GCP_OK) return st;
    if ((want & GCP_IMPL_PLAIN) || grad_scale) return GCP_E_UNSUPPORTED;
    void* Gs[3];
    for (int k = 0; k < 3; ++k) Gs[k] = (want & GCP_WANT_GRAD) ? G[k] : fac_ptr(s, s->L.G, k);
    hipError_t eb = build_current_table(s, X_t);
    if (eb != hipSuccess) return hip_status(eb);
    SampledCall c = sampled_call(s, X_t, A, s_t, want & (GCP_WANT_LOSS | GCP_WANT_GRAD),
                                 (want & GCP_WANT_LOSS) ? loss : s->ws + s->L.loss, Gs,
                                 (want & GCP_WANT_GRAD) ? g_s : s->ws + s->L.gs);
    if (s->ev_used + 2 <= (int)s->ev.size()) {
      c.ev_begin = s->ev[s->ev_used];
      c.ev_end = s->ev[s->ev_used + 1];
      s->ev_used += 2;
    }
    hipError_t es = sampled_run(c);
    if (es == hipSuccess) es = add_model_history(s, A, c.want, c.loss_out, c.G, nullptr);
    if (es == hipSuccess && (want & GCP_WANT_LOSS)) es = d2_fix_loss(s, c.loss_out);
    return hip_status(es);
  }
  gcp_status st = check_dense_slice(s, X_t);
  if (st != GCP_OK) return st;
  const bool plain = want & GCP_IMPL_PLAIN;
  if (plain && s->L.plain_bytes == 0) return GCP_E_STATE;
  if (plain && grad_scale) return GCP_E_UNSUPPORTED;
  DenseCall c = base_call(s);
  c.want = want & (GCP_WANT_LOSS | GCP_WANT_GRAD);
  c.X[0] = X_t->vals;
  c.S[0] = s_t;
  fill_window(s, c);
  for (int k = 0; k < 3; ++k) {
    c.A[k] = A[k];
    c.G[k] = (want & GCP_WANT_GRAD) ? G[k] : nullptr;
  }
  c.gs = (want & GCP_WANT_GRAD) ? g_s : nullptr;
  c.loss_out = (want & GCP_WANT_LOSS) ? loss : nullptr;
  c.grad_scale = grad_scale;
  if ((want & GCP_WANT_GRAD) == 0) {
    // the fused kernel always forms gradients; route them to scratch
    for (int k = 0; k < 3; ++k) c.G[k] = fac_ptr(s, s->L.G, k);
    if (d4) c.G[2] = s->ws + s->L.G34;
    c.gs = s->ws + s->L.gs;
  }
  c.merged34 = d4;
  if (!plain && s->ev_used + 2 <= (int)s->ev.size()) {
    c.ev_begin = s->ev[s->ev_used];
    c.ev_end = s->ev[s->ev_used + 1];
    s->ev_used += 2;
  }
  const bool ident = use_identity(s, c.want, plain, grad_scale);
  if (ident) c.loss = kGaussianId;
  hipError_t e = plain ? dense_plain_run(c, s->ws + s->L.plain, s->L.plain_bytes) : dense_fused_run(c);
  if (e == hipSuccess && d4)
    e = finish_four_way(s, A_in, c.want, c.lam, c.loss_out, (want & GCP_WANT_GRAD) ? G_in[2] : nullptr,
                        (want & GCP_WANT_GRAD) ? G_in[3] : nullptr, grad_scale);
  if (e == hipSuccess && ident) e = identity_terms(s, c);
  if (e == hipSuccess) e = add_model_history(s, A, c.want, c.loss_out, c.G, grad_scale);
  if (e == hipSuccess && (want & GCP_WANT_LOSS)) e = d2_fix_loss(s, c.loss_out);
  return hip_status(e);
}

// Algorithm 3 on a COO slice: sampled weight gradients over X_t alone (a new
// call number each), Algorithm 5's estimates over draws fixed for the solve.
static hipError_t coo_weight_sgd(gcp_stream* s, const gcp_slice* X_t, void* s_t) {
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  void* G[3] = {fac_ptr(s, s->L.G, 0), fac_ptr(s, s->L.G, 1), fac_ptr(s, s->L.G, 2)};
  void* gs = s->ws + s->L.gs;
  void* loss = s->ws + s->L.loss;
  const TsgdCall tc = tsgd_call(s, nullptr, A, s_t, s->status);
  auto estimate = [&]() {
    SampledCall c = sampled_call(s, X_t, A, s_t, kWantLoss, loss, G, gs, (int64_t)weight_estimate_call(s->t));
    c.ns = 1;             // the weight problem has no history term
    c.lam = 0.0;
    c.p = s->p.p_est;
    c.q = s->p.q_est;
    return sampled_run(c);
  };
  hipError_t e = build_current_table(s, X_t);
  if (e == hipSuccess) e = tsgd_sampled_begin(tc);
  if (e == hipSuccess) e = estimate();
  if (e == hipSuccess) e = tsgd_sampled_decide(tc, loss, 1);
  for (int ep = 0; ep < s->p.kappa_w && e == hipSuccess; ++ep) {
    for (int it = 0; it < s->p.tau_w && e == hipSuccess; ++it) {
      SampledCall c = sampled_call(s, X_t, A, s_t, kWantGrad, loss, G, gs);
      c.ns = 1;
      c.lam = 0.0;
      e = sampled_run(c);
      if (e == hipSuccess) e = tsgd_sampled_step(tc, gs);
    }
    if (e == hipSuccess) e = estimate();
    if (e == hipSuccess) e = tsgd_sampled_decide(tc, loss, 0);
  }
  return e;
}

gcp_status gcp_solve_st(gcp_stream* s, const gcp_slice* X_t, void* s_t) {
  if (!s || !s_t) return GCP_E_ARG;
  const bool coo = s->p.slice_kind == GCP_SLICE_COO;
  if (s->p.tsolve == GCP_TSOLVE_LS && (coo || s->p.loss != GCP_LOSS_GAUSSIAN)) return GCP_E_UNSUPPORTED;
  gcp_status st = coo ? check_coo_slice(s, X_t) : check_dense_slice(s, X_t);
  if (st != GCP_OK) return st;
  if (coo) return hip_status(coo_weight_sgd(s, X_t, s_t));
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  if (four_way(s)) {
    // the weights see the model through the merged modes 3 and 4
    const void* A4[4] = {A[0], A[1], A[2], fac_ptr(s, s->L.A, 3)};
    hipError_t em = kernel_factors(s, A4, A, s->L.A34, s->p.rank);
    if (em != hipSuccess) return hip_status(em);
  }
  if (s->p.tsolve == GCP_TSOLVE_SGD) {
    const void* X = X_t->vals;
    if (bits_stream(s)) {
      // the weights' solve reads X_t as FP32 values
      float* xf = reinterpret_cast<float*>(s->ws + s->L.xf);
      hipError_t e = unpack_bits_run(X, xf, (int64_t)s->dims[0] * s->dims[1], s->dims[2], s->st);
      if (e != hipSuccess) return hip_status(e);
      X = xf;
    }
    return hip_status(tsgd_run(tsgd_call(s, X, A, s_t, s->status)));
  }
  return hip_status(ls_solve_run(s->dims[0], s->dims[1], s->dims[2], s->p.rank, s->p.dtype, X_t->vals, A, s->p.mu,
                                 s->p.lower, s_t, s->ws + s->L.ls, s->status, s->st));
}

gcp_status gcp_solve_st_info(gcp_stream* s, double* F, double* alpha, int64_t* iters, int32_t* epochs,
                             uint64_t* rolled) {
  if (!s) return GCP_E_ARG;
  if (s->p.tsolve != GCP_TSOLVE_SGD) return GCP_E_STATE;
  TsgdState h;
  hipError_t e = hipMemcpyAsync(&h, s->ws + s->L.tsgd, sizeof(h), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return GCP_E_DEVICE;
  if (F) *F = h.F;
  if (alpha) *alpha = h.alpha;
  if (iters) *iters = h.i;
  if (epochs) *epochs = h.epoch;
  if (rolled) *rolled = h.rolled;
  return GCP_OK;
}

namespace {

// One full dense gradient of the stream's objective at its current factors
// into the gradient scratch (data term, window, history, regularisation).
static hipError_t dense_grad_step(gcp_stream* s, const gcp_slice* X_t, const void* s_t) {
  DenseCall c = base_call(s);
  c.want = kWantGrad;
  c.X[0] = X_t->vals;
  c.S[0] = s_t;
  fill_window(s, c);
  for (int k = 0; k < 3; ++k) {
    c.A[k] = fac_ptr(s, s->L.A, k);
    c.G[k] = fac_ptr(s, s->L.G, k);
  }
  c.gs = s->ws + s->L.gs;
  const void* A4[4] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2),
                       four_way(s) ? fac_ptr(s, s->L.A, 3) : nullptr};
  hipError_t e = hipSuccess;
  if (four_way(s)) {
    e = kernel_factors(s, A4, c.A, s->L.A34, s->p.rank);
    c.G[2] = s->ws + s->L.G34;
    c.merged34 = 1;
  }
  const bool ident = use_identity(s, kWantGrad, false, nullptr);
  if (ident) c.loss = kGaussianId;
  if (e == hipSuccess) e = dense_fused_run(c);
  if (e == hipSuccess && four_way(s))
    e = finish_four_way(s, A4, kWantGrad, c.lam, nullptr, fac_ptr(s, s->L.G, 2), fac_ptr(s, s->L.G, 3), nullptr);
  if (e == hipSuccess && ident) e = identity_terms(s, c);
  if (e == hipSuccess) e = add_model_history(s, c.A, kWantGrad, nullptr, c.G, nullptr);
  if (e == hipSuccess) e = d2_clear_fixed_grad(s);
  return e;
}

// The objective Algorithm 4 compares (no mu/2 ||s_t||^2 term) into `loss`.
static hipError_t dense_objective(gcp_stream* s, const gcp_slice* X_t, const void* s_t, void* loss) {
  DenseCall c = base_call(s);
  c.want = kWantLoss;
  c.mu = 0.0;
  c.X[0] = X_t->vals;
  c.S[0] = s_t;
  fill_window(s, c);
  for (int k = 0; k < 3; ++k) {
    c.A[k] = fac_ptr(s, s->L.A, k);
    c.G[k] = fac_ptr(s, s->L.G, k);   // formed by the kernel, not used
  }
  c.gs = s->ws + s->L.gs;
  c.loss_out = loss;
  const void* A4[4] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2),
                       four_way(s) ? fac_ptr(s, s->L.A, 3) : nullptr};
  hipError_t e = hipSuccess;
  if (four_way(s)) {
    e = kernel_factors(s, A4, c.A, s->L.A34, s->p.rank);
    c.G[2] = s->ws + s->L.G34;
    c.merged34 = 1;
  }
  if (e == hipSuccess) e = dense_fused_run(c);
  if (e == hipSuccess && four_way(s)) e = finish_four_way(s, A4, kWantLoss, c.lam, loss, nullptr, nullptr, nullptr);
  if (e == hipSuccess) e = add_model_history(s, c.A, kWantLoss, loss, c.G, nullptr);
  if (e == hipSuccess) e = d2_fix_loss(s, loss);
  return e;
}

// One sampled gradient of a COO stream's objective into the gradient scratch
// (a new call number).
static hipError_t coo_grad_step(gcp_stream* s, const gcp_slice* X_t, const void* s_t) {
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  void* G[3] = {fac_ptr(s, s->L.G, 0), fac_ptr(s, s->L.G, 1), fac_ptr(s, s->L.G, 2)};
  SampledCall c = sampled_call(s, X_t, A, s_t, kWantGrad, s->ws + s->L.loss, G, s->ws + s->L.gs);
  hipError_t e = sampled_run(c);
  if (e == hipSuccess) e = add_model_history(s, A, kWantGrad, nullptr, G, nullptr);
  if (e == hipSuccess) e = d2_clear_fixed_grad(s);
  return e;
}

// Algorithm 5's estimate for the factor solver of time step t: p_est and
// q_est draws per slice under a call number fixed for the solve, exact
// history and factor regulariser, no weight regulariser.
static hipError_t coo_objective(gcp_stream* s, const gcp_slice* X_t, const void* s_t, void* loss) {
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  void* G[3] = {fac_ptr(s, s->L.G, 0), fac_ptr(s, s->L.G, 1), fac_ptr(s, s->L.G, 2)};
  SampledCall c = sampled_call(s, X_t, A, s_t, kWantLoss, loss, G, s->ws + s->L.gs,
                               (int64_t)factor_estimate_call(s->t));
  c.p = s->p.p_est;
  c.q = s->p.q_est;
  c.mu = 0.0;
  hipError_t e = sampled_run(c);
  if (e == hipSuccess) e = add_model_history(s, A, kWantLoss, loss, G, nullptr);
  if (e == hipSuccess) e = d2_fix_loss(s, loss);
  return e;
}

// Algorithm 4's epochs with every decision on the device.
static hipError_t factor_epochs(gcp_stream* s, const gcp_slice* X_t, const void* s_t) {
  const gcp_params& p = s->p;
  const bool coo = p.slice_kind == GCP_SLICE_COO;
  FacState* st = reinterpret_cast<FacState*>(s->ws + s->L.fac);
  void* loss = s->ws + s->L.fac + 256;
  const int64_t n = (int64_t)s->L.fac_elems;
  const int dt = p.dtype == GCP_F64;
  auto objective = [&]() { return coo ? coo_objective(s, X_t, s_t, loss) : dense_objective(s, X_t, s_t, loss); };
  hipError_t e = objective();
  if (e == hipSuccess) e = fac_begin_run(dt, st, loss, p.tol_f, s->st);
  for (int ep = 0; ep < p.kappa_f && e == hipSuccess; ++ep) {
    for (int it = 0; it < p.tau_f && e == hipSuccess; ++it) {
      e = coo ? coo_grad_step(s, X_t, s_t) : dense_grad_step(s, X_t, s_t);
      if (e == hipSuccess)
        e = fac_step_run(dt, adam_elems(s), s->ws + s->L.A, s->ws + s->L.G, s->ws + s->L.u, s->ws + s->L.v, st, p.beta1,
                         p.beta2, p.adam_eps, p.lower, s->st);
    }
    if (e == hipSuccess) e = objective();
    if (e == hipSuccess)
      e = fac_end_epoch_run(dt, n, s->ws + s->L.A, s->ws + s->L.u, s->ws + s->L.v, s->ws + s->L.Ao,
                            s->ws + s->L.uo, s->ws + s->L.vo, st, loss, p.tau_f, p.tol_f, p.beta1, p.beta2, s->st);
  }
  return e;
}

}  // namespace

gcp_status gcp_factor_info(gcp_stream* s, double* F, double* alpha, int64_t* iters, int32_t* epochs,
                           uint64_t* rolled) {
  if (!s) return GCP_E_ARG;
  if (s->p.kappa_f == 0) return GCP_E_STATE;
  FacState h;
  hipError_t e = hipMemcpyAsync(&h, s->ws + s->L.fac, sizeof(h), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return GCP_E_DEVICE;
  if (F) *F = h.F;
  if (alpha) *alpha = h.alpha;
  if (iters) *iters = h.i;
  if (epochs) *epochs = h.epoch;
  if (rolled) *rolled = h.rolled;
  return GCP_OK;
}

gcp_status gcp_update_factors(gcp_stream* s, const gcp_slice* X_t, const void* s_t) {
  if (!s || !s_t) return GCP_E_ARG;
  const bool coo = s->p.slice_kind == GCP_SLICE_COO;
  gcp_status st = coo ? check_coo_slice(s, X_t) : check_dense_slice(s, X_t);
  if (st != GCP_OK) return st;
  const gcp_params& p = s->p;
  hipError_t e = coo ? build_current_table(s, X_t) : hipSuccess;
  for (int it = 0; it < (p.kappa_f > 0 ? 0 : p.tau_f) && e == hipSuccess; ++it) {
    if (coo) {
      e = coo_grad_step(s, X_t, s_t);
      if (e != hipSuccess) break;
      const double n = (double)(s->adam_i + 1);
      const double alpha_t = p.alpha_f * sqrt(1.0 - pow(p.beta2, n)) / (1.0 - pow(p.beta1, n));
      e = adam_run(p.dtype, adam_elems(s), s->ws + s->L.A, s->ws + s->L.G, s->ws + s->L.u,
                   s->ws + s->L.v, alpha_t, p.beta1, p.beta2, p.adam_eps, p.lower, s->st);
      s->adam_i += 1;
      continue;
    }
    e = dense_grad_step(s, X_t, s_t);
    if (e != hipSuccess) break;
    const double n = (double)(s->adam_i + 1);
    const double alpha_t = p.alpha_f * sqrt(1.0 - pow(p.beta2, n)) / (1.0 - pow(p.beta1, n));
    e = adam_run(p.dtype, adam_elems(s), s->ws + s->L.A, s->ws + s->L.G, s->ws + s->L.u,
                 s->ws + s->L.v, alpha_t, p.beta1, p.beta2, p.adam_eps, p.lower, s->st);
    s->adam_i += 1;
  }
  if (p.kappa_f > 0 && e == hipSuccess) e = factor_epochs(s, X_t, s_t);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ws + s->L.Aold, s->ws + s->L.A, s->L.fac_elems * s->es, hipMemcpyDeviceToDevice, s->st);
  // a failed launch leaves the window, the time index and the slot stamps
  // as they were
  if (e != hipSuccess) return hip_status(e);
  // reservoir window update (Algorithm 1), then t <- t+1
  int slot = -1;
  if (p.window > 0) {
    if (s->nwin < p.window) {
      slot = s->nwin;
    } else {
      uint64_t j = splitmix64(p.seed ^ (uint64_t)s->t) % (uint64_t)s->t + 1;
      if (j <= (uint64_t)p.window) slot = (int)(j - 1);
    }
  }
  if (slot >= 0) {
    if (model_hist(s))
      ;   // only s_t and t are kept
    else if (coo)
      e = store_coo_slot(s, slot, X_t);
    else
      e = store_dense_slot(s, slot, X_t->vals);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->ws + s->L.shist + (size_t)slot * p.rank * s->es, s_t, p.rank * s->es,
                         hipMemcpyDeviceToDevice, s->st);
    if (e == hipSuccess) e = hist_set_stamp_run(reinterpret_cast<int64_t*>(s->ws + s->L.stamps), slot, s->t, s->st);
    if (e != hipSuccess) return hip_status(e);
    if (s->nwin == slot) s->nwin += 1;
    s->slot_t[slot] = s->t;
  }
  s->t += 1;
  return GCP_OK;
}

gcp_status gcp_slice_loss(gcp_stream* s, const gcp_slice* X, const void* s_x, double* sum_f, double* sum_sq) {
  if (!s || !s_x) return GCP_E_ARG;
  if (s->p.slice_kind == GCP_SLICE_COO) return GCP_E_UNSUPPORTED;
  gcp_status st = check_dense_slice(s, X);
  if (st != GCP_OK) return st;
  const void* Xv = X->vals;
  if (bits_stream(s)) {
    // the loss and the norm over the slice as FP32 0/1 values
    float* xf = reinterpret_cast<float*>(s->ws + s->L.xf);
    hipError_t eu = unpack_bits_run(Xv, xf, (int64_t)s->dims[0] * s->dims[1], s->dims[2], s->st);
    if (eu != hipSuccess) return hip_status(eu);
    Xv = xf;
  }
  DenseCall c = base_call(s);
  c.xbits = 0;
  c.want = kWantLoss;
  c.lam = 0.0;
  c.mu = 0.0;
  c.X[0] = Xv;
  c.S[0] = s_x;
  c.ns = 1;
  for (int k = 0; k < 3; ++k) {
    c.A[k] = fac_ptr(s, s->L.A, k);
    c.G[k] = fac_ptr(s, s->L.G, k);   // formed by the kernel, not used
  }
  c.gs = s->ws + s->L.gs;
  c.loss_out = s->ws + s->L.loss;
  double* sq = reinterpret_cast<double*>(s->ws + s->L.loss + 64);
  hipError_t e = hipSuccess;
  if (four_way(s)) {
    const void* A4[4] = {c.A[0], c.A[1], c.A[2], fac_ptr(s, s->L.A, 3)};
    e = kernel_factors(s, A4, c.A, s->L.A34, s->p.rank);
    c.G[2] = s->ws + s->L.G34;
    c.merged34 = 1;
  }
  if (e == hipSuccess) e = dense_fused_run(c);
  if (e == hipSuccess) e = sumsq_run(s->p.dtype == GCP_F64, Xv, (int64_t)s->omega, s->ws + s->L.metric, sq, s->st);
  double f = 0.0, q = 0.0;
  if (e == hipSuccess) {
    if (s->p.dtype == GCP_F64) {
      e = hipMemcpyAsync(&f, s->ws + s->L.loss, 8, hipMemcpyDeviceToHost, s->st);
    } else {
      float f32 = 0.f;
      e = hipMemcpyAsync(&f32, s->ws + s->L.loss, 4, hipMemcpyDeviceToHost, s->st);
      if (e == hipSuccess) e = hipStreamSynchronize(s->st);
      f = f32;
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&q, sq, 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return GCP_E_DEVICE;
  if (sum_f) *sum_f = f;
  if (sum_sq) *sum_sq = q;
  return GCP_OK;
}

gcp_status gcp_local_loss(gcp_stream* s, const gcp_slice* X, const void* s_x, double* out) {
  if (!out) return GCP_E_ARG;
  double f = 0.0, q = 0.0;
  gcp_status st = gcp_slice_loss(s, X, s_x, &f, &q);
  if (st != GCP_OK) return st;
  *out = q > 0.0 ? f / q : std::numeric_limits<double>::quiet_NaN();
  return GCP_OK;
}

gcp_status gcp_ktensor_score(gcp_stream* s, const void* w_a, const void* const* B, const void* w_b, int32_t rank_b,
                             double* score) {
  if (!s || !w_a || !B || !B[0] || !B[1] || (!B[2] && s->p.d >= 3) || (!B[3] && s->p.d == 4) || !w_b || !score)
    return GCP_E_ARG;
  if (rank_b < 1 || rank_b > GCP_MAX_RANK) return GCP_E_ARG;
  if (four_way(s) && rank_b > s->p.rank) return GCP_E_ARG;   // the merged reference rows use the stream's scratch
  const int Ra = s->p.rank, Rb = rank_b;
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  const int dt = s->p.dtype == GCP_F64;
  // matrix slices: the reference's two factors go to internal modes 0 and 2
  const void* Bi[3] = {B[0], s->p.d == 2 ? metrics_ones(s->ws + s->L.metric) : B[1], s->p.d == 2 ? B[1] : B[2]};
  hipError_t e = hipSuccess;
  if (four_way(s)) {
    // four-way: both K-tensors through merged modes 3 and 4.  A merged
    // column is a3 (x) a4, whose norm and inner products are the products of
    // the modes' ones, so the per-mode product of cosines is unchanged.
    const void* A4[4] = {A[0], A[1], A[2], fac_ptr(s, s->L.A, 3)};
    e = kernel_factors(s, A4, A, s->L.A34, Ra);
    if (e == hipSuccess) e = kernel_factors(s, B, Bi, s->L.B34, Rb);
  }
  if (e == hipSuccess) e = cross_run(dt, A, Bi, s->dims, Ra, Rb, s->ws + s->L.metric, s->st);
  std::vector<double> h((size_t)3 * Ra * Rb + 3 * Ra + 3 * Rb);
  std::vector<double> wa(Ra), wb(Rb);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), cross_results(s->ws + s->L.metric), h.size() * 8, hipMemcpyDeviceToHost, s->st);
  if (dt) {
    if (e == hipSuccess) e = hipMemcpyAsync(wa.data(), w_a, Ra * 8, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(wb.data(), w_b, Rb * 8, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  } else {
    std::vector<float> fa(Ra), fb(Rb);
    if (e == hipSuccess) e = hipMemcpyAsync(fa.data(), w_a, Ra * 4, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(fb.data(), w_b, Rb * 4, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    for (int r = 0; r < Ra; ++r) wa[r] = fa[r];
    for (int q = 0; q < Rb; ++q) wb[q] = fb[q];
  }
  if (e != hipSuccess) return GCP_E_DEVICE;
  const double* C = h.data();
  const double* Na = C + (size_t)3 * Ra * Rb;
  const double* Nb = Na + 3 * Ra;
  // component weights with the column norms moved in, then pair scores
  std::vector<double> xi(Ra), eta(Rb);
  for (int r = 0; r < Ra; ++r) {
    xi[r] = std::fabs(wa[r]);
    for (int k = 0; k < 3; ++k) xi[r] *= std::sqrt(Na[k * Ra + r]);
  }
  for (int q = 0; q < Rb; ++q) {
    eta[q] = std::fabs(wb[q]);
    for (int k = 0; k < 3; ++k) eta[q] *= std::sqrt(Nb[k * Rb + q]);
  }
  struct Pair { double v; int r, q; };
  std::vector<Pair> P;
  P.reserve((size_t)Ra * Rb);
  for (int r = 0; r < Ra; ++r)
    for (int q = 0; q < Rb; ++q) {
      double cg = 1.0;
      for (int k = 0; k < 3; ++k) {
        const double na = std::sqrt(Na[k * Ra + r]), nb = std::sqrt(Nb[k * Rb + q]);
        cg *= (na > 0 && nb > 0) ? std::fabs(C[((size_t)k * Ra + r) * Rb + q]) / (na * nb) : 0.0;
      }
      const double big = std::max(xi[r], eta[q]);
      const double pen = 1.0 - (big > 0 ? std::fabs(xi[r] - eta[q]) / big : 0.0);
      P.push_back({cg * pen, r, q});
    }
  std::sort(P.begin(), P.end(), [](const Pair& a, const Pair& b) {
    if (a.v != b.v) return a.v > b.v;
    if (a.r != b.r) return a.r < b.r;
    return a.q < b.q;
  });
  std::vector<char> ua(Ra, 0), ub(Rb, 0);
  double total = 0.0;
  int matched = 0;
  for (const Pair& x : P) {
    if (ua[x.r] || ub[x.q]) continue;
    ua[x.r] = ub[x.q] = 1;
    total += x.v;
    if (++matched == std::min(Ra, Rb)) break;
  }
  *score = total / Rb;
  return GCP_OK;
}

gcp_status gcp_get_factors(gcp_stream* s, void* const* A_out) {
  if (!s || !A_out || !A_out[0] || !A_out[1] || (!A_out[2] && s->p.d >= 3) || (s->p.d == 4 && !A_out[3]))
    return GCP_E_ARG;
  hipError_t e = hipSuccess;
  for (int k = 0; k < (s->p.d == 2 ? 2 : s->p.d) && e == hipSuccess; ++k) {
    const int ki = int_mode(s, k);
    const size_t rows = four_way(s) && k >= 2 ? (size_t)s->d4[k - 2] : (size_t)s->dims[ki];
    e = hipMemcpyAsync(A_out[k], fac_ptr(s, s->L.A, ki), rows * s->p.rank * s->es, hipMemcpyDeviceToDevice, s->st);
  }
  return hip_status(e);
}

gcp_status gcp_factor_ptr(gcp_stream* s, int32_t k, void** ptr) {
  if (!s || !ptr || k < 0 || k > (s->p.d == 4 ? 3 : 2)) return GCP_E_ARG;
  *ptr = fac_ptr(s, s->L.A, int_mode(s, k));
  return GCP_OK;
}

gcp_status gcp_stream_info(gcp_stream* s, int64_t* t, int32_t* n_window, int64_t* adam_iter, int64_t* slot_times,
                           int64_t* sample_call) {
  if (!s) return GCP_E_ARG;
  if (sample_call) *sample_call = s->sample_call;
  if (t) *t = s->t;
  if (n_window) *n_window = s->nwin;
  if (adam_iter) {
    if (s->p.kappa_f > 0) {
      // the factor epochs keep the index on the device
      FacState h;
      hipError_t e = hipMemcpyAsync(&h, s->ws + s->L.fac, sizeof(h), hipMemcpyDeviceToHost, s->st);
      if (e == hipSuccess) e = hipStreamSynchronize(s->st);
      if (e != hipSuccess) return GCP_E_DEVICE;
      *adam_iter = h.i;
    } else {
      *adam_iter = s->adam_i;
    }
  }
  if (slot_times)
    for (int h = 0; h < s->p.window; ++h) slot_times[h] = h < s->nwin ? s->slot_t[h] : 0;
  return GCP_OK;
}

gcp_status gcp_stream_sync(gcp_stream* s) {
  if (!s) return GCP_E_ARG;
  if (hipStreamSynchronize(s->st) != hipSuccess) return GCP_E_DEVICE;
  int word = 0;
  if (hipMemcpy(&word, s->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return GCP_E_DEVICE;
  if (word != 0) {
    if (hipMemset(s->status, 0, sizeof(int)) != hipSuccess) return GCP_E_DEVICE;
    return GCP_E_NUMERIC;
  }
  return GCP_OK;
}

gcp_status gcp_dump_samples(gcp_stream* s, const gcp_slice* X_t, int32_t h_index, int64_t call, int32_t* coords,
                            float* weights, int64_t cap, int64_t* n) {
  if (!s || !coords || !weights || !n) return GCP_E_ARG;
  if (s->p.slice_kind != GCP_SLICE_COO) return GCP_E_UNSUPPORTED;
  if (call < 0 || h_index < 0 || h_index > (model_hist(s) ? 0 : s->nwin)) return GCP_E_ARG;
  const int64_t total = s->p.p + s->p.q;
  if (cap < total) return GCP_E_ARG;
  gcp_status st = check_coo_slice(s, X_t);
  if (st != GCP_OK) return st;
  hipError_t e = h_index == 0 ? build_current_table(s, X_t) : hipSuccess;
  if (e != hipSuccess) return hip_status(e);
  const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
  void* G[3] = {fac_ptr(s, s->L.G, 0), fac_ptr(s, s->L.G, 1), fac_ptr(s, s->L.G, 2)};
  SampledCall c = sampled_call(s, X_t, A, s->ws + s->L.gs, kWantGrad, s->ws + s->L.loss, G, s->ws + s->L.gs, call);
  *n = total;
  return hip_status(sampled_dump_run(c, h_index, coords, weights));
}

gcp_status gcp_kernel_timing(gcp_stream* s, int32_t enable, int32_t capacity) {
  if (!s || capacity < 0) return GCP_E_ARG;
  if (hipStreamSynchronize(s->st) != hipSuccess) return GCP_E_DEVICE;
  for (hipEvent_t e : s->ev) hipEventDestroy(e);
  s->ev.clear();
  s->ev_used = 0;
  if (!enable) return GCP_OK;
  s->ev.resize((size_t)capacity * 2);
  for (auto& e : s->ev)
    if (hipEventCreate(&e) != hipSuccess) return GCP_E_DEVICE;
  return GCP_OK;
}

gcp_status gcp_kernel_time(gcp_stream* s, double* total_ms, int64_t* count) {
  if (!s || !total_ms || !count) return GCP_E_ARG;
  double tot = 0.0;
  for (int i = 0; i + 1 < s->ev_used; i += 2) {
    if (hipEventSynchronize(s->ev[i + 1]) != hipSuccess) return GCP_E_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]) != hipSuccess) return GCP_E_DEVICE;
    tot += ms;
  }
  *total_ms = tot;
  *count = s->ev_used / 2;
  s->ev_used = 0;
  return GCP_OK;
}

gcp_status gcp_stream_destroy(gcp_stream* s) {
  if (!s) return GCP_E_ARG;
  hipStreamSynchronize(s->st);
  for (hipEvent_t e : s->ev) hipEventDestroy(e);
  delete s;
  return GCP_OK;
}

const char* gcp_status_string(gcp_status st) {
  switch (st) {
    case GCP_OK: return "ok";
    case GCP_E_ARG: return "invalid argument";
    case GCP_E_SHAPE: return "shape mismatch";
    case GCP_E_ALIGN: return "misaligned pointer";
    case GCP_E_STATE: return "invalid stream state";
    case GCP_E_WORKSPACE: return "workspace too small";
    case GCP_E_DEVICE: return "HIP runtime error";
    case GCP_E_NUMERIC: return "non-finite value or failed pivot on the device";
    case GCP_E_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

}  // extern "C"

// ------------------------------------------------------------- autotuner
namespace {

bool cache_lookup(const char* path, const char* key, int* value) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[400];
    int v = 0;
    if (sscanf(line, "%399[^=]= %d", k, &v) == 2) {
      size_t n = strlen(k);
      while (n > 0 && k[n - 1] == ' ') k[--n] = 0;
      if (strcmp(k, key) == 0) {
        *value = v;
        found = true;
      }
    }
  }
  fclose(f);
  return found;
}

bool is_plan_target(int v) {
  for (int i = 0; i < kNumPlanTargets; ++i)
    if (kPlanTargets[i] == v) return true;
  return false;
}

// Shape bucket of the tuned work plan: the tile build (loss, rank tile,
// h-tiles, copy width), the (i1, i2) pair count by powers of two and I3 by
// 64-entry groups.
void tune_key(char* key, size_t n, const char* arch, const gcp_stream* s) {
  const long pairs = (long)s->dims[0] * s->dims[1];
  int lp = 0;
  while ((1L << (lp + 1)) <= pairs) ++lp;
  const int ns = 1 + s->nwin;
  snprintf(key, n, "%s loss%d rt%d nh%d dma%d pairs2^%d i3x64:%d", arch, s->p.loss, s->p.rank > 16 ? 32 : 16,
           (ns + 15) / 16, copy_mode(s->L.rp3, s->dims[2]), lp, (s->dims[2] + 63) / 64);
}

}  // namespace

extern "C" gcp_status gcp_autotune(gcp_stream* s, const gcp_slice* X_t, const char* cache_path, int32_t* chosen) {
  if (!s) return GCP_E_ARG;
  if (s->p.slice_kind != GCP_SLICE_DENSE || s->p.dtype != GCP_F32 || four_way(s)) return GCP_E_UNSUPPORTED;
  gcp_status st = check_dense_slice(s, X_t);
  if (st != GCP_OK) return st;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return GCP_E_DEVICE;
  char key[400];
  tune_key(key, sizeof key, prop.gcnArchName, s);
  int best = 0;
  if (cache_lookup(cache_path, key, &best) && is_plan_target(best)) {
    s->plan_target = best;
    if (chosen) *chosen = best;
    return GCP_OK;
  }
  DenseCall c = base_call(s);
  c.want = kWantLoss | kWantGrad;
  c.kernel = 2;
  c.X[0] = X_t->vals;
  c.S[0] = s->ws + s->L.shist;   // any R weights will do for timing
  if (s->nwin == 0) c.S[0] = s->ws + s->L.A;
  fill_window(s, c);
  for (int k = 0; k < 3; ++k) {
    c.A[k] = fac_ptr(s, s->L.A, k);
    c.G[k] = fac_ptr(s, s->L.G, k);
  }
  c.gs = s->ws + s->L.gs;
  c.loss_out = s->ws + s->L.loss;
  if (!mfma_supported(c.R, c.ns, 0)) return GCP_E_UNSUPPORTED;
  // one warm-up call per candidate plan, then single calls timed
  // round-robin over the candidates (clock drift falls on all alike); the
  // lowest median call decides
  constexpr int kReps = 7;
  hipEvent_t ev[kNumPlanTargets][kReps][2] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < kNumPlanTargets && e == hipSuccess; ++i)
    for (int r = 0; r < kReps && e == hipSuccess; ++r)
      for (int k = 0; k < 2 && e == hipSuccess; ++k)
        if ((e = hipEventCreate(&ev[i][r][k])) != hipSuccess) ev[i][r][k] = nullptr;
  for (int i = 0; i < kNumPlanTargets && e == hipSuccess; ++i) {
    c.plan_target = kPlanTargets[i];
    e = dense_fused_run(c);
  }
  for (int r = 0; r < kReps && e == hipSuccess; ++r)
    for (int i = 0; i < kNumPlanTargets && e == hipSuccess; ++i) {
      c.plan_target = kPlanTargets[i];
      e = hipEventRecord(ev[i][r][0], s->st);
      if (e == hipSuccess) e = dense_fused_run(c);
      if (e == hipSuccess) e = hipEventRecord(ev[i][r][1], s->st);
    }
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  float best_ms = 1e30f;
  best = kDefaultPlanTarget;
  for (int i = 0; i < kNumPlanTargets && e == hipSuccess; ++i) {
    float t[kReps];
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = hipEventElapsedTime(&t[r], ev[i][r][0], ev[i][r][1]);
    if (e != hipSuccess) break;
    std::sort(t, t + kReps);
    if (t[kReps / 2] < best_ms) {
      best_ms = t[kReps / 2];
      best = kPlanTargets[i];
    }
  }
  for (int i = 0; i < kNumPlanTargets; ++i)
    for (int r = 0; r < kReps; ++r)
      for (int k = 0; k < 2; ++k)
        if (ev[i][r][k]) hipEventDestroy(ev[i][r][k]);
  if (e != hipSuccess) return GCP_E_DEVICE;
  s->plan_target = best;
  if (chosen) *chosen = best;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s = %d\n", key, best);
      fclose(f);
    }
  }
  return GCP_OK;
}

// ------------------------------------------------- allocation-free entry
namespace {

// Partial sums of gcp_loss_grad_static: one array per GPU, held until the
// process ends.  Host code never hands `scratch` itself to a kernel (its
// host-side name is not a device address); each device's address is taken
// once with hipGetSymbolAddress while that device is current.
__device__ __align__(256) char scratch[GCP_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mutex;
void* g_scratch_dev[256];

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

extern "C" gcp_status gcp_loss_grad_static(const gcp_params* p, const gcp_slice* X_t, int32_t n_hist,
                                           const void* X_hist, const void* s_hist, const int64_t* t_hist,
                                           int64_t t, const void* const* A, const void* s_t, uint32_t want,
                                           void* loss, void* const* G, void* g_s, hipStream_t stream) {
  gcp_status st = check_params(p);
  if (st != GCP_OK) return st;
  if (p->d != 3 || p->slice_kind != GCP_SLICE_DENSE || p->hist != GCP_HIST_SLICES) return GCP_E_UNSUPPORTED;
  if (p->flags & (GCP_FLAG_PLAIN_SCRATCH | GCP_FLAG_GAUSS_IDENTITY)) return GCP_E_UNSUPPORTED;
  if (!X_t || X_t->kind != GCP_SLICE_DENSE || !X_t->vals || !A || !A[0] || !A[1] || !A[2] || !s_t)
    return GCP_E_ARG;
  if (n_hist < 0 || n_hist > p->window) return GCP_E_ARG;
  if (n_hist > 0 && (!X_hist || !s_hist || !t_hist)) return GCP_E_ARG;
  if ((want & ~(uint32_t)(GCP_WANT_LOSS | GCP_WANT_GRAD)) || !(want & (GCP_WANT_LOSS | GCP_WANT_GRAD)))
    return GCP_E_ARG;
  if ((want & GCP_WANT_LOSS) && !loss) return GCP_E_ARG;
  if ((want & GCP_WANT_GRAD) && (!G || !G[0] || !G[1] || !G[2] || !g_s)) return GCP_E_ARG;
  if (!aligned16(X_t->vals) || (n_hist > 0 && !aligned16(X_hist))) return GCP_E_ALIGN;
  for (int h = 0; h < n_hist; ++h)
    if (t_hist[h] >= t) return GCP_E_ARG;
  const int I1 = (int)p->dims[0], I2 = (int)p->dims[1], I3 = (int)p->dims[2], R = p->rank;
  const size_t es = p->dtype == GCP_F64 ? 8 : 4;
  const size_t omega = (size_t)I1 * I2 * I3;
  // scratch: status word | partial sums | (gradient-free calls) a sink for
  // the gradients the fused kernel always forms
  const size_t part = dense_fused_part_bytes(I1, I2, I3, R, p->dtype);
  const size_t sink = (want & GCP_WANT_GRAD) ? 0 : align_up((size_t)(I1 + I2 + I3 + 1) * R * es, 256);
  if (256 + align_up(part, 256) + sink > (size_t)GCP_STATIC_SCRATCH_BYTES) return GCP_E_WORKSPACE;
  void* vbase = nullptr;
  if (scratch_address(&vbase) != hipSuccess) return GCP_E_DEVICE;
  char* base = static_cast<char*>(vbase);
  DenseCall c;
  memset(&c, 0, sizeof(c));
  c.I1 = I1;
  c.I2 = I2;
  c.I3 = I3;
  c.R = R;
  c.loss = p->loss;
  c.dtype = p->dtype;
  c.lam = p->lambda;
  c.mu = p->mu;
  c.status = reinterpret_cast<int*>(base);   // written by kernels, never read back
  c.part = base + 256;
  c.part_bytes = align_up(part, 256);
  c.stream = stream;
  c.kernel = (p->flags & GCP_FLAG_KERNEL_VALU) ? 1 : ((p->flags & GCP_FLAG_KERNEL_MFMA) ? 2 : 0);
  c.want = want;
  c.X[0] = X_t->vals;
  c.S[0] = s_t;
  c.c[0] = 1.0;
  // window: n_hist slices one after another, rows of pitch I3
  c.ring = X_hist;
  c.ring_pitch = (size_t)I3;
  c.ring_stride = omega;
  c.shist = s_hist;
  c.omega = omega;
  for (int h = 0; h < n_hist; ++h) {
    c.X[h + 1] = static_cast<const char*>(X_hist) + (size_t)h * omega * es;
    c.S[h + 1] = static_cast<const char*>(s_hist) + (size_t)h * R * es;
    c.c[h + 1] = p->w * pow(p->theta, (double)(t - t_hist[h]));
  }
  c.ns = n_hist + 1;
  char* sk = base + 256 + align_up(part, 256);
  size_t off = 0;
  for (int k = 0; k < 3; ++k) {
    c.A[k] = A[k];
    if (want & GCP_WANT_GRAD) {
      c.G[k] = G[k];
    } else {
      c.G[k] = sk + off;
      off += (size_t)p->dims[k] * R * es;
    }
  }
  c.gs = (want & GCP_WANT_GRAD) ? g_s : static_cast<void*>(sk + off);
  c.loss_out = (want & GCP_WANT_LOSS) ? loss : nullptr;
  return hip_status(dense_fused_run(c));
}

extern "C" gcp_status gcp_probe_gather(const void* A1, const void* A2, const void* A3, int64_t I1, int64_t I2,
                                       int64_t I3, int32_t rank, int64_t ndraws, uint64_t seed, void* records,
                                       hipStream_t hip_stream) {
  if (!A1 || !A2 || !A3 || !records || ndraws < 0) return GCP_E_ARG;
  if (I1 < 1 || I2 < 1 || I3 < 1 || I1 > (1 << 30) || I2 > (1 << 30) || I3 > (1 << 30)) return GCP_E_SHAPE;
  if (rank < 1 || rank > GCP_MAX_RANK) return GCP_E_ARG;
  if (ndraws == 0) return GCP_OK;
  return hip_status(gather_probe_run(static_cast<const float*>(A1), static_cast<const float*>(A2),
                                     static_cast<const float*>(A3), (int)I1, (int)I2, (int)I3, rank, ndraws, seed,
                                     records, hip_stream));
}

// Per-bucket autotuning for a set of streams about to be batched: the
// largest stream (by window entries) of each shape bucket is tuned (or read
// from the cache) and every stream of the bucket takes its plan.
extern "C" gcp_status gcp_batch_autotune(gcp_stream* const* streams, const gcp_batch_io* io, int32_t n,
                                         const char* cache_path, int32_t* buckets) {
  if (!streams || !io || n < 1) return GCP_E_ARG;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return GCP_E_DEVICE;
  std::vector<std::string> keys(n);
  for (int i = 0; i < n; ++i) {
    if (!streams[i] || !io[i].X_t) return GCP_E_ARG;
    char key[400];
    tune_key(key, sizeof key, prop.gcnArchName, streams[i]);
    keys[i] = key;
  }
  // the batch's key: its shape buckets, sorted, with their counts (FNV-1a)
  std::vector<std::string> sorted = keys;
  std::sort(sorted.begin(), sorted.end());
  uint64_t h = 1469598103934665603ull;
  for (const std::string& k : sorted)
    for (unsigned char ch : k + "\n") h = (h ^ ch) * 1099511628211ull;
  const int nb = (int)(std::unique(sorted.begin(), sorted.end()) - sorted.begin());
  if (buckets) *buckets = nb;
  char bkey[160];
  snprintf(bkey, sizeof bkey, "%s batch n%d buckets%d %016llx", prop.gcnArchName, n, nb, (unsigned long long)h);
  int best = 0;
  if (cache_lookup(cache_path, bkey, &best) && is_plan_target(best)) {
    for (int i = 0; i < n; ++i) streams[i]->batch_plan_target = best;
    return GCP_OK;
  }
  // one batch per candidate plan, each on a scratch workspace of its own size
  // (the registered outputs are written and later overwritten); then single
  // objective+gradient calls timed round-robin over the candidates, so that
  // clock and thermal drift falls on all of them alike, and the median call
  // of each candidate decides
  constexpr int kCands = 4, kReps = 9;
  const int cands[kCands] = {512, 1024, 2048, 4096};
  gcp_batch* bs[kCands] = {};
  void* wss[kCands] = {};
  best = kBatchPlanTarget;
  gcp_status st = GCP_OK;
  for (int c = 0; c < kCands && st == GCP_OK; ++c) {
    for (int i = 0; i < n; ++i) streams[i]->batch_plan_target = cands[c];
    size_t bytes = 0;
    st = gcp_batch_workspace_size(streams, n, &bytes);
    if (st == GCP_OK && hipMalloc(&wss[c], bytes) != hipSuccess) {
      wss[c] = nullptr;
      st = GCP_E_DEVICE;
    }
    if (st == GCP_OK) st = gcp_batch_create(streams, io, n, wss[c], bytes, streams[0]->st, &bs[c]);
    if (st == GCP_OK) st = gcp_batch_loss_grad(bs[c], GCP_WANT_LOSS | GCP_WANT_GRAD);   // warm-up
  }
  hipEvent_t ev[kCands][kReps][2] = {};
  for (int c = 0; c < kCands && st == GCP_OK; ++c)
    for (int r = 0; r < kReps && st == GCP_OK; ++r)
      for (int k = 0; k < 2 && st == GCP_OK; ++k)
        if (hipEventCreate(&ev[c][r][k]) != hipSuccess) {
          ev[c][r][k] = nullptr;
          st = GCP_E_DEVICE;
        }
  for (int r = 0; r < kReps && st == GCP_OK; ++r)
    for (int c = 0; c < kCands && st == GCP_OK; ++c) {
      if (hipEventRecord(ev[c][r][0], streams[0]->st) != hipSuccess) st = GCP_E_DEVICE;
      if (st == GCP_OK) st = gcp_batch_loss_grad(bs[c], GCP_WANT_LOSS | GCP_WANT_GRAD);
      if (st == GCP_OK && hipEventRecord(ev[c][r][1], streams[0]->st) != hipSuccess) st = GCP_E_DEVICE;
    }
  if (st == GCP_OK && hipStreamSynchronize(streams[0]->st) != hipSuccess) st = GCP_E_DEVICE;
  float best_ms = 1e30f;
  for (int c = 0; c < kCands && st == GCP_OK; ++c) {
    float t[kReps];
    for (int r = 0; r < kReps && st == GCP_OK; ++r)
      if (hipEventElapsedTime(&t[r], ev[c][r][0], ev[c][r][1]) != hipSuccess) st = GCP_E_DEVICE;
    if (st != GCP_OK) break;
    std::sort(t, t + kReps);
    if (t[kReps / 2] < best_ms) {
      best_ms = t[kReps / 2];
      best = cands[c];
    }
  }
  for (int c = 0; c < kCands; ++c)
    for (int r = 0; r < kReps; ++r)
      for (int k = 0; k < 2; ++k)
        if (ev[c][r][k]) hipEventDestroy(ev[c][r][k]);
  if (hipStreamSynchronize(streams[0]->st) != hipSuccess && st == GCP_OK) st = GCP_E_DEVICE;
  for (int c = 0; c < kCands; ++c) {
    if (bs[c]) gcp_batch_destroy(bs[c]);
    if (wss[c]) hipFree(wss[c]);
  }
  for (int i = 0; i < n; ++i) streams[i]->batch_plan_target = best;
  if (st != GCP_OK) return st;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s = %d\n", bkey, best);
      fclose(f);
    }
  }
  return GCP_OK;
}

// --------------------------------------------------------------- batching
struct gcp_batch {
  std::vector<gcp_stream*> streams;
  std::vector<gcp_batch_io> io;   // registered buffers, per stream
  hipStream_t st;
  char* ws;
  BatchRun run_out;     // reduce writes the registered outputs
  BatchRun run_step;    // reduce writes each stream's gradient scratch
  int* status;
  int tau_f;
  int kappa_f;
};

namespace {

struct BatchLayout {
  size_t desc_out, desc_step, state, items, counter, outstart, facstart, cpystart, parts, total;
  int nitems;
  std::vector<size_t> part_off;
  std::vector<MfmaPlan> plans;
};

// The batch's own lane streams and fork/join events (lane 0 is the caller's).
void batch_release_lanes(BatchRun& r) {
  for (int l = 1; l < kBatchLanes; ++l) {
    if (r.lane[l]) {
      hipStreamSynchronize(r.lane[l]);
      hipStreamDestroy(r.lane[l]);
    }
    if (r.join[l]) hipEventDestroy(r.join[l]);
    r.lane[l] = nullptr;
    r.join[l] = nullptr;
  }
  if (r.fork) hipEventDestroy(r.fork);
  r.fork = nullptr;
}

size_t mfma_part_bytes(const MfmaPlan& m, int I1, int I2, int I3, int R) {
  size_t b = 0;
  b = align_up(b + (size_t)m.nb2 * I1 * R * 4, 256);
  b = align_up(b + (size_t)m.nb1 * I2 * R * 4, 256);
  b = align_up(b + (size_t)m.nwg * I3 * R * 4, 256);
  b = align_up(b + (size_t)m.nwg * R * 4, 256);
  b = align_up(b + (size_t)m.nwg * 4, 256);
  return b;
}

gcp_status batch_check(gcp_stream* const* streams, int32_t n) {
  if (!streams || n < 1) return GCP_E_ARG;
  for (int i = 0; i < n; ++i) {
    const gcp_stream* s = streams[i];
    if (!s) return GCP_E_ARG;
    if (s->p.slice_kind != GCP_SLICE_DENSE || s->p.dtype != GCP_F32) return GCP_E_UNSUPPORTED;
    if (s->p.rank > 32 || s->p.window > 31) return GCP_E_UNSUPPORTED;
    if (model_hist(s)) return GCP_E_UNSUPPORTED;   // batches run the stored-slice history
    if (s->p.loss > GCP_LOSS_BERNOULLI_LOGIT) return GCP_E_UNSUPPORTED;   // batch tiles: the first three losses
    if (s->p.kappa_f != streams[0]->p.kappa_f) return GCP_E_ARG;   // epochs run in lockstep
    if (s->p.d != 3) return GCP_E_UNSUPPORTED;
    if (s->p.tau_f != streams[0]->p.tau_f) return GCP_E_ARG;
    if (s->st != streams[0]->st) return GCP_E_ARG;
  }
  return GCP_OK;
}

BatchLayout batch_layout(gcp_stream* const* streams, int32_t n) {
  BatchLayout L;
  size_t off = 0;
  L.nitems = 0;
  for (int i = 0; i < n; ++i) {
    const gcp_stream* s = streams[i];
    L.plans.push_back(mfma_plan(s->dims[0], s->dims[1], s->dims[2], kBatchTileWaves, s->batch_plan_target));
    L.nitems += L.plans.back().nwg;
  }
  L.desc_out = off; off = align_up(off + n * sizeof(BatchDesc), 256);
  L.desc_step = off; off = align_up(off + n * sizeof(BatchDesc), 256);
  L.state = off; off = align_up(off + n * sizeof(BatchState), 256);
  L.items = off; off = align_up(off + (size_t)L.nitems * sizeof(int2), 256);
  static_assert(kBatchVariants <= 48, "work counters precede the status word");
  L.counter = off; off += 256;
  L.outstart = off; off = align_up(off + n * sizeof(int64_t), 256);
  L.facstart = off; off = align_up(off + n * sizeof(int64_t), 256);
  L.cpystart = off; off = align_up(off + n * sizeof(int64_t), 256);
  L.parts = off;
  for (int i = 0; i < n; ++i) {
    const gcp_stream* s = streams[i];
    L.part_off.push_back(off);
    off = align_up(off + mfma_part_bytes(L.plans[i], s->dims[0], s->dims[1], s->dims[2], s->p.rank), 256);
  }
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

gcp_status gcp_batch_workspace_size(gcp_stream* const* streams, int32_t n, size_t* bytes) {
  if (!bytes) return GCP_E_ARG;
  gcp_status st = batch_check(streams, n);
  if (st != GCP_OK) return st;
  *bytes = batch_layout(streams, n).total;
  return GCP_OK;
}

gcp_status gcp_batch_create(gcp_stream* const* streams, const gcp_batch_io* io, int32_t n, void* workspace,
                            size_t ws_bytes, hipStream_t hip_stream, gcp_batch** out) {
  if (!out || !io || !workspace) return GCP_E_ARG;
  *out = nullptr;
  gcp_status st = batch_check(streams, n);
  if (st != GCP_OK) return st;
  if (((uintptr_t)workspace & 255u) != 0) return GCP_E_ALIGN;
  BatchLayout L = batch_layout(streams, n);
  if (ws_bytes < L.total) return GCP_E_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    if (!io[i].X_t || !io[i].s_t) return GCP_E_ARG;
    if (!aligned16(io[i].X_t)) return GCP_E_ALIGN;
  }
  char* ws = static_cast<char*>(workspace);
  std::vector<BatchDesc> dout(n), dstep(n);
  std::vector<BatchState> state(n);
  std::vector<int64_t> outstart(n), facstart(n), cpystart(n);
  std::vector<std::pair<double, int>> order;
  int64_t nout = 0, nfac = 0, ncpy = 0;
  for (int i = 0; i < n; ++i) {
    gcp_stream* s = streams[i];
    const MfmaPlan& m = L.plans[i];
    const int I1 = s->dims[0], I2 = s->dims[1], I3 = s->dims[2], R = s->p.rank;
    BatchDesc d;
    memset(&d, 0, sizeof(d));
    d.Xt = static_cast<const float*>(io[i].X_t);
    d.st = static_cast<const float*>(io[i].s_t);
    d.ring = reinterpret_cast<float*>(s->ws + s->L.ring);
    d.shist = reinterpret_cast<float*>(s->ws + s->L.shist);
    d.A = reinterpret_cast<float*>(s->ws + s->L.A);
    d.Aold = reinterpret_cast<float*>(s->ws + s->L.Aold);
    d.u = reinterpret_cast<float*>(s->ws + s->L.u);
    d.v = reinterpret_cast<float*>(s->ws + s->L.v);
    d.Gs = reinterpret_cast<float*>(s->ws + s->L.G);
    char* pb = ws + L.part_off[i];
    size_t o = 0;
    d.G1p = reinterpret_cast<float*>(pb + o); o = align_up(o + (size_t)m.nb2 * I1 * R * 4, 256);
    d.G2p = reinterpret_cast<float*>(pb + o); o = align_up(o + (size_t)m.nb1 * I2 * R * 4, 256);
    d.G3p = reinterpret_cast<float*>(pb + o); o = align_up(o + (size_t)m.nwg * I3 * R * 4, 256);
    d.gsp = reinterpret_cast<float*>(pb + o); o = align_up(o + (size_t)m.nwg * R * 4, 256);
    d.lossp = reinterpret_cast<float*>(pb + o);
    d.omega = (int64_t)s->omega;
    d.rp3 = (int64_t)s->L.rp3;
    d.rstride = (int64_t)s->L.slot_elems;
    d.fac_elems = (int64_t)s->L.fac_elems;
    d.fac_off1 = (int64_t)s->L.fac_off[1];
    d.fac_off2 = (int64_t)s->L.fac_off[2];
    d.I1 = I1; d.I2 = I2; d.I3 = I3; d.R = R; d.H = s->p.window; d.loss = s->p.loss;
    d.variant = batch_variant(s->p.loss, R, s->p.window, s->L.rp3, I3);
    d.tb1 = m.tb1; d.tb2 = m.tb2; d.nb1 = m.nb1; d.nb2 = m.nb2; d.nblocks = m.nblocks; d.nwg = m.nwg;
    d.w = s->p.w; d.theta = s->p.theta; d.lam = (float)s->p.lambda; d.mu = (float)s->p.mu;
    d.lower = s->p.lower == -INFINITY ? -INFINITY : (float)s->p.lower;
    d.alpha = s->p.alpha_f; d.beta1 = (float)s->p.beta1; d.beta2 = (float)s->p.beta2;
    d.beta1d = s->p.beta1; d.beta2d = s->p.beta2;
    d.eps = (float)s->p.adam_eps;
    d.seed = s->p.seed;
    if (s->p.kappa_f > 0) {
      d.fac = reinterpret_cast<FacState*>(s->ws + s->L.fac);
      d.Ao = reinterpret_cast<float*>(s->ws + s->L.Ao);
      d.uo = reinterpret_cast<float*>(s->ws + s->L.uo);
      d.vo = reinterpret_cast<float*>(s->ws + s->L.vo);
      d.tol_f = s->p.tol_f;
    }
    // step descriptor: gradients into the stream's scratch
    dstep[i] = d;
    for (int k = 0; k < 3; ++k) dstep[i].outG[k] = reinterpret_cast<float*>(fac_ptr(s, s->L.G, k));
    dstep[i].outgs = reinterpret_cast<float*>(s->ws + s->L.gs);
    dstep[i].outloss = reinterpret_cast<float*>(s->ws + s->L.loss);
    // output descriptor: registered outputs, scratch where none was given
    dout[i] = dstep[i];
    for (int k = 0; k < 3; ++k)
      if (io[i].G[k]) dout[i].outG[k] = static_cast<float*>(io[i].G[k]);
    if (io[i].g_s) dout[i].outgs = static_cast<float*>(io[i].g_s);
    if (io[i].loss) dout[i].outloss = static_cast<float*>(io[i].loss);
    BatchState& b = state[i];
    memset(&b, 0, sizeof(b));
    b.t = s->t;
    b.adam_i = s->adam_i;
    b.nwin = s->nwin;
    b.pending_slot = -1;
    for (int h = 0; h < s->nwin; ++h) b.slot_t[h] = s->slot_t[h];
    outstart[i] = nout;
    nout += (int64_t)(I1 + I2 + I3 + 1) * R + 1;
    facstart[i] = nfac;
    nfac += (int64_t)s->L.fac_elems;
    cpystart[i] = ncpy;
    ncpy += (int64_t)s->L.fac_elems + (int64_t)s->omega + R;
    const double cost = (double)s->omega * (s->p.window + 1) * (R > 16 ? 2.0 : 1.0) / m.nwg;
    order.push_back({cost, i});
  }
  // work list grouped by tile variant (one persistent launch each); inside a
  // variant the most expensive streams come first, so each launch ends with
  // short items
  std::vector<int> var(n);
  for (int i = 0; i < n; ++i)
    var[i] = batch_variant(streams[i]->p.loss, streams[i]->p.rank, streams[i]->p.window, streams[i]->L.rp3,
                           streams[i]->dims[2]);
  std::sort(order.begin(), order.end(), [&](const std::pair<double, int>& x, const std::pair<double, int>& y) {
    if (var[x.second] != var[y.second]) return var[x.second] < var[y.second];
    return x.first > y.first;
  });
  std::vector<int2> items;
  int vbegin[kBatchVariants], vend[kBatchVariants];
  for (int v = 0; v < kBatchVariants; ++v) vbegin[v] = vend[v] = 0;
  for (auto& pr : order) {
    const int v = var[pr.second];
    if (vend[v] == vbegin[v]) vbegin[v] = vend[v] = (int)items.size();
    for (int w = 0; w < L.plans[pr.second].nwg; ++w) items.push_back(make_int2(pr.second, w));
    vend[v] = (int)items.size();
  }
  hipError_t e = hipMemcpy(ws + L.desc_out, dout.data(), n * sizeof(BatchDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.desc_step, dstep.data(), n * sizeof(BatchDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.state, state.data(), n * sizeof(BatchState), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.outstart, outstart.data(), n * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.facstart, facstart.data(), n * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.cpystart, cpystart.data(), n * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(ws + L.counter, 0, 256);
  if (e != hipSuccess) return GCP_E_DEVICE;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  gcp_batch* b = new (std::nothrow) gcp_batch();
  if (!b) return GCP_E_ARG;
  b->streams.assign(streams, streams + n);
  b->io.assign(io, io + n);
  b->st = hip_stream;
  b->ws = ws;
  b->status = reinterpret_cast<int*>(ws + L.counter) + 48;   // after the kBatchVariants counters
  b->tau_f = streams[0]->p.tau_f;
  b->kappa_f = streams[0]->p.kappa_f;
  BatchRun r;
  r.desc = reinterpret_cast<const BatchDesc*>(ws + L.desc_out);
  r.state = reinterpret_cast<BatchState*>(ws + L.state);
  r.items = reinterpret_cast<const int2*>(ws + L.items);
  r.nitems = (int)items.size();
  r.counter = reinterpret_cast<int*>(ws + L.counter);
  r.nstreams = n;
  r.outstart = reinterpret_cast<const int64_t*>(ws + L.outstart);
  r.nout = nout;
  r.facstart = reinterpret_cast<const int64_t*>(ws + L.facstart);
  r.nfac = nfac;
  r.cpystart = reinterpret_cast<const int64_t*>(ws + L.cpystart);
  r.ncpy = ncpy;
  // variants present, most expensive first, each given to the lane (HIP
  // stream) with the least work so far
  std::vector<std::pair<double, int>> vcost;
  for (int v = 0; v < kBatchVariants; ++v) {
    r.vbegin[v] = vbegin[v];
    r.vend[v] = vend[v];
    r.vlane[v] = 0;
    // the rank-16 single-tile variant fits two workgroups per compute unit
    const int per_cu = batch_variant_r16(v) ? 2 : 1;
    r.vgrid[v] = std::max(1, std::min(per_cu * cus, vend[v] - vbegin[v]));
    if (vend[v] > vbegin[v]) vcost.push_back({0.0, v});
  }
  for (auto& pr : order)
    for (auto& vc : vcost)
      if (vc.second == var[pr.second]) vc.first += pr.first * L.plans[pr.second].nwg;
  std::sort(vcost.begin(), vcost.end(), [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
    return x.first != y.first ? x.first > y.first : x.second < y.second;
  });
  r.nvar = (int)vcost.size();
  r.nlanes = std::max(1, std::min(r.nvar, kBatchLanes));
  double lane_load[kBatchLanes] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < r.nvar; ++i) {
    r.vorder[i] = vcost[i].second;
    int best = 0;
    for (int l = 1; l < r.nlanes; ++l)
      if (lane_load[l] < lane_load[best]) best = l;
    r.vlane[vcost[i].second] = best;
    lane_load[best] += vcost[i].first;
  }
  r.lane[0] = hip_stream;
  for (int l = 1; l < kBatchLanes; ++l) r.lane[l] = nullptr;
  r.fork = nullptr;
  for (int l = 0; l < kBatchLanes; ++l) r.join[l] = nullptr;
  bool lanes_ok = hipEventCreateWithFlags(&r.fork, hipEventDisableTiming) == hipSuccess;
  for (int l = 1; l < r.nlanes && lanes_ok; ++l)
    lanes_ok = hipStreamCreateWithFlags(&r.lane[l], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&r.join[l], hipEventDisableTiming) == hipSuccess;
  r.status = b->status;
  r.stream = hip_stream;
  if (!lanes_ok) {
    b->run_out = r;
    batch_release_lanes(b->run_out);
    delete b;
    return GCP_E_DEVICE;
  }
  b->run_out = r;
  b->run_step = r;
  b->run_step.desc = reinterpret_cast<const BatchDesc*>(ws + L.desc_step);
  *out = b;
  return GCP_OK;
}

gcp_status gcp_batch_loss_grad(gcp_batch* b, uint32_t want) {
  if (!b) return GCP_E_ARG;
  want &= (GCP_WANT_LOSS | GCP_WANT_GRAD);
  if (!want) return GCP_E_ARG;
  return hip_status(batch_grad_run(b->run_out, (int)want));
}

gcp_status gcp_batch_update_factors(gcp_batch* b) {
  if (!b) return GCP_E_ARG;
  hipError_t e = hipSuccess;
  if (b->kappa_f > 0) {
    // Algorithm 4's epochs, every decision on the device (per stream):
    // objective at the start, then per epoch tau_f gradient + ADAM steps and
    // the keep-or-undo test on the objective
    const int obj = kWantLoss | kWantObjective;
    e = batch_grad_run(b->run_step, obj);
    if (e == hipSuccess) e = batch_fac_begin_run(b->run_step);
    for (int ep = 0; ep < b->kappa_f && e == hipSuccess; ++ep) {
      for (int it = 0; it < b->tau_f && e == hipSuccess; ++it) {
        e = batch_grad_run(b->run_step, kWantGrad);
        if (e == hipSuccess) e = batch_fac_step_run(b->run_step);
      }
      if (e == hipSuccess) e = batch_grad_run(b->run_step, obj);
      if (e == hipSuccess) e = batch_fac_end_run(b->run_step, b->tau_f);
    }
  } else {
    for (int it = 0; it < b->tau_f && e == hipSuccess; ++it) {
      e = batch_grad_run(b->run_step, kWantGrad);
      if (e == hipSuccess) e = batch_adam_run(b->run_step);
    }
  }
  if (e == hipSuccess) e = batch_window_run(b->run_step);
  return hip_status(e);
}

gcp_status gcp_batch_solve_st(gcp_batch* b) {
  if (!b) return GCP_E_ARG;
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < b->streams.size() && e == hipSuccess; ++i) {
    gcp_stream* s = b->streams[i];
    const void* A[3] = {fac_ptr(s, s->L.A, 0), fac_ptr(s, s->L.A, 1), fac_ptr(s, s->L.A, 2)};
    if (s->p.tsolve == GCP_TSOLVE_SGD) {
      TsgdCall c = tsgd_call(s, b->io[i].X_t, A, const_cast<void*>(b->io[i].s_t), b->status);
      c.stream = b->st;
      e = tsgd_run(c);
      continue;
    }
    if (s->p.loss != GCP_LOSS_GAUSSIAN) continue;
    e = ls_solve_run(s->dims[0], s->dims[1], s->dims[2], s->p.rank, s->p.dtype, b->io[i].X_t, A, s->p.mu,
                     s->p.lower, const_cast<void*>(b->io[i].s_t), s->ws + s->L.ls, b->status, b->st);
  }
  return hip_status(e);
}

gcp_status gcp_batch_step(gcp_batch* b) {
  gcp_status st = gcp_batch_solve_st(b);
  if (st != GCP_OK) return st;
  return gcp_batch_update_factors(b);
}

gcp_status gcp_batch_sync_streams(gcp_batch* b) {
  if (!b) return GCP_E_ARG;
  const int n = (int)b->streams.size();
  std::vector<BatchState> state(n);
  if (hipStreamSynchronize(b->st) != hipSuccess) return GCP_E_DEVICE;
  if (hipMemcpy(state.data(), b->run_out.state, n * sizeof(BatchState), hipMemcpyDeviceToHost) != hipSuccess)
    return GCP_E_DEVICE;
  int word = 0;
  if (hipMemcpy(&word, b->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return GCP_E_DEVICE;
  for (int i = 0; i < n; ++i) {
    gcp_stream* s = b->streams[i];
    s->t = state[i].t;
    s->adam_i = state[i].adam_i;
    s->nwin = state[i].nwin;
    for (int h = 0; h < s->nwin; ++h) s->slot_t[h] = state[i].slot_t[h];
    // the device copy of the stamps follows (the host array lives on)
    if (s->nwin > 0 && hipMemcpy(s->ws + s->L.stamps, s->slot_t.data(), (size_t)s->nwin * 8,
                                 hipMemcpyHostToDevice) != hipSuccess)
      return GCP_E_DEVICE;
  }
  if (word != 0) {
    if (hipMemset(b->status, 0, sizeof(int)) != hipSuccess) return GCP_E_DEVICE;
    return GCP_E_NUMERIC;
  }
  return GCP_OK;
}

gcp_status gcp_batch_destroy(gcp_batch* b) {
  if (!b) return GCP_E_ARG;
  hipStreamSynchronize(b->st);
  batch_release_lanes(b->run_out);
  delete b;
  return GCP_OK;
}

}  // extern "C"
