"""Python handle over the C ABI.  PyTorch supplies device memory (the
workspace, outputs) and the HIP stream; every computation runs in the
library's kernels.  Function names mirror the C calls."""
from __future__ import annotations

import ctypes
import math
from ctypes import byref, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p
from typing import List, Optional, Sequence

import torch

from . import _native as N


def _ptr(t: Optional[torch.Tensor]):
    return c_void_p(0 if t is None else t.data_ptr())


def _ptr_array(ts: Sequence[torch.Tensor], n: int = 0):
    """Device pointers of ts, padded with NULL to n entries (matrix slices
    pass two factors where the C ABI takes three)."""
    arr = (c_void_p * max(n, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _dense_slice(x: torch.Tensor) -> N.GcpSlice:
    """A dense slice of values, or (int32 words) a bit-packed binary slice:
    rows of ceil(I3/32) words, entry i3 is bit i3 % 32 of word i3 // 32."""
    if not x.is_contiguous():
        raise ValueError("dense slices must be contiguous (row-major)")
    kind = N.SLICE_BITS if x.dtype == torch.int32 else N.SLICE_DENSE
    return N.GcpSlice(kind, 0, x.data_ptr(), None, 0)


def _slice(x) -> N.GcpSlice:
    """A dense tensor, or a (coords int32 [nnz,3], vals [nnz]) pair sorted by
    row-major linear index."""
    if isinstance(x, torch.Tensor):
        return _dense_slice(x)
    coords, vals = x
    if coords.dtype != torch.int32 or not coords.is_contiguous() or not vals.is_contiguous():
        raise ValueError("COO slices need contiguous int32 coords [nnz,3] and values [nnz]")
    return N.GcpSlice(N.SLICE_COO, 0, vals.data_ptr(), coords.data_ptr(), int(vals.numel()))


def make_params(dims, rank: int, window: int, loss: str, *, w=1.0, theta=1.0,
                lam=0.0, mu=0.0, lower=-math.inf, alpha_f=1e-3, beta1=0.9,
                beta2=0.999, adam_eps=1e-8, tau_f=1, seed=0,
                dtype=torch.float32, plain=False, kernel: str = "auto",
                slice_kind: str = "dense", max_nnz: int = 0, p: int = 0, q: int = 0,
                sampled_atomic: bool = False, hist: str = "slices", tsolve: str = "ls",
                tau_w: int = 100, kappa_w: int = 20, alpha_w: float = 1.0,
                tol_w: float = -math.inf, kappa_f: int = 0, tol_f: float = -math.inf,
                p_est: int = 0, q_est: int = 0, gauss_identity: bool = False) -> N.GcpParams:
    lib = N.load()
    n_p, n_q = p, q
    p = N.GcpParams()
    lib.gcp_params_default(byref(p))
    p.slice_kind = {"coo": N.SLICE_COO, "bits": N.SLICE_BITS}.get(slice_kind, N.SLICE_DENSE)
    p.max_nnz, p.p, p.q = int(max_nnz), int(n_p), int(n_q)
    p.d = len(dims)
    for k, n in enumerate(list(dims)[:4]):
        p.dims[k] = int(n)
    if p.d == 2:
        p.dims[2] = 1           # matrix slices: I3 = 1, fixed third factor
    p.rank = int(rank)
    p.window = int(window)
    p.loss = N.LOSS_IDS[loss]
    p.dtype = N.F64 if dtype == torch.float64 else N.F32
    p.flags = (N.FLAG_PLAIN_SCRATCH if plain else 0) | {
        "auto": 0, "valu": N.FLAG_KERNEL_VALU, "mfma": N.FLAG_KERNEL_MFMA}[kernel] | (
        N.FLAG_SAMPLED_ATOMIC if sampled_atomic else 0) | (N.FLAG_GAUSS_IDENTITY if gauss_identity else 0)
    p.hist = {"slices": N.HIST_SLICES, "model": N.HIST_MODEL}[hist]
    p.w, p.theta, p.lam, p.mu, p.lower = float(w), float(theta), float(lam), float(mu), float(lower)
    p.alpha_f, p.beta1, p.beta2, p.adam_eps = float(alpha_f), float(beta1), float(beta2), float(adam_eps)
    p.tau_f = int(tau_f)
    p.tsolve = {"ls": N.TSOLVE_LS, "sgd": N.TSOLVE_SGD}[tsolve]
    p.tau_w, p.kappa_w, p.alpha_w, p.tol_w = int(tau_w), int(kappa_w), float(alpha_w), float(tol_w)
    p.kappa_f, p.tol_f = int(kappa_f), float(tol_f)
    p.p_est, p.q_est = int(p_est), int(q_est)
    p.seed = int(seed) & ((1 << 64) - 1)
    return p


def gcp_workspace_size(params: N.GcpParams) -> int:
    lib = N.load()
    n = c_size_t(0)
    N.check(lib.gcp_workspace_size(byref(params), byref(n)), "gcp_workspace_size")
    return int(n.value)


class Stream:
    """One streaming-GCP state on one device (Algorithm 1's loop state)."""

    def __init__(self, dims, rank: int, window: int, loss: str, A0: Sequence[torch.Tensor],
                 X_hist: Sequence[torch.Tensor] = (), s_hist: Optional[torch.Tensor] = None,
                 t_hist: Optional[Sequence[int]] = None, **kw):
        self.lib = N.load()
        self.dtype = A0[0].dtype
        self.device = A0[0].device
        if self.device.type != "cuda":
            raise ValueError("gcpstream runs on the GPU only: pass device tensors")
        self.params = make_params(dims, rank, window, loss, dtype=self.dtype, **kw)
        self.coo = self.params.slice_kind == N.SLICE_COO
        self.dims = tuple(int(n) for n in dims)
        self.rank = int(rank)
        self.window = int(window)
        self.loss = loss
        nbytes = gcp_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.hip_stream = torch.cuda.current_stream(self.device)
        # the model-difference history keeps no slices: its window is given
        # by the weights and time stamps alone
        n_hist = len(X_hist) if len(X_hist) else (len(t_hist) if t_hist is not None else 0)
        slices = (N.GcpSlice * max(1, n_hist))()
        for h, x in enumerate(X_hist):
            slices[h] = _slice(x)
        th = (c_int64 * max(1, n_hist))(*(list(t_hist) if t_hist is not None else []))
        A0c = [a.contiguous() for a in A0]
        sh = s_hist.contiguous() if s_hist is not None and n_hist > 0 else None
        handle = c_void_p(0)
        N.check(self.lib.gcp_stream_init(byref(self.params), _ptr_array(A0c, 3), n_hist, slices,
                                         _ptr(sh), th, _ptr(self.workspace), nbytes,
                                         c_void_p(self.hip_stream.cuda_stream), byref(handle)),
                "gcp_stream_init")
        self._keep = (A0c, sh, list(X_hist))  # alive until the copies have run
        # (the copies run on the caller's stream; tensors stay referenced)
        self.handle = handle

    # -- calls ----------------------------------------------------------
    def loss_grad(self, X_t: torch.Tensor, A: Sequence[torch.Tensor], s_t: torch.Tensor,
                  want_loss: bool = True, want_grad: bool = True, plain: bool = False,
                  out=None, grad_scale: Optional[torch.Tensor] = None):
        want = (N.WANT_LOSS if want_loss else 0) | (N.WANT_GRAD if want_grad else 0)
        if plain:
            want |= N.IMPL_PLAIN
        dev, dt = self.device, self.dtype
        if out is None:
            loss = torch.empty(1, dtype=dt, device=dev)
            G = [torch.empty(n, self.rank, dtype=dt, device=dev) for n in self.dims]
            g_s = torch.empty(self.rank, dtype=dt, device=dev)
        else:
            loss, G, g_s = out
        sl = _slice(X_t)
        Ac = [a.contiguous() for a in A]
        N.check(self.lib.gcp_loss_grad_scaled(self.handle, byref(sl), _ptr_array(Ac, 3),
                                              _ptr(s_t.contiguous()), want, _ptr(grad_scale),
                                              _ptr(loss), _ptr_array(G, 3), _ptr(g_s)),
                "gcp_loss_grad")
        return loss, G, g_s

    def dump_samples(self, X_t, h: int = 0, call: int = 0):
        """The sampler's draws for slice h (0: X_t) at call number `call`:
        (coords [n, 3] int32, weights [n]) on the device (COO streams)."""
        n_all = int(self.params.p + self.params.q)
        coords = torch.empty(n_all, 3, dtype=torch.int32, device=self.device)
        weights = torch.empty(n_all, dtype=torch.float32, device=self.device)
        n = c_int64(0)
        sl = _slice(X_t)
        N.check(self.lib.gcp_dump_samples(self.handle, byref(sl), int(h), int(call), _ptr(coords),
                                          _ptr(weights), n_all, byref(n)), "gcp_dump_samples")
        return coords[: n.value], weights[: n.value]

    def solve_st(self, X_t: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        s = out if out is not None else torch.empty(self.rank, dtype=self.dtype, device=self.device)
        sl = _slice(X_t)
        N.check(self.lib.gcp_solve_st(self.handle, byref(sl), _ptr(s)), "gcp_solve_st")
        return s

    def solve_info(self) -> dict:
        """State of the last SGD temporal solve (synchronises the stream)."""
        F, alpha = c_double(0.0), c_double(0.0)
        iters, epochs, rolled = c_int64(0), c_int32(0), c_uint64(0)
        N.check(self.lib.gcp_solve_st_info(self.handle, byref(F), byref(alpha), byref(iters), byref(epochs),
                                           byref(rolled)), "gcp_solve_st_info")
        return {"F": F.value, "alpha": alpha.value, "iters": iters.value, "epochs": epochs.value,
                "rolled": [bool(rolled.value >> e & 1) for e in range(epochs.value)]}

    def factor_info(self) -> dict:
        """State of the factor epochs of the last update (synchronises the stream)."""
        F, alpha = c_double(0.0), c_double(0.0)
        iters, epochs, rolled = c_int64(0), c_int32(0), c_uint64(0)
        N.check(self.lib.gcp_factor_info(self.handle, byref(F), byref(alpha), byref(iters), byref(epochs),
                                         byref(rolled)), "gcp_factor_info")
        return {"F": F.value, "alpha": alpha.value, "iters": iters.value, "epochs": epochs.value,
                "rolled": [bool(rolled.value >> e & 1) for e in range(epochs.value)]}

    def slice_loss(self, X: torch.Tensor, s_x: torch.Tensor):
        """(sum_i f(x_i, m_i), ||X||_F^2) of a dense slice under the current
        factors with weights s_x (synchronises the stream)."""
        f, q = c_double(0.0), c_double(0.0)
        sl = _dense_slice(X)
        N.check(self.lib.gcp_slice_loss(self.handle, byref(sl), _ptr(s_x.contiguous()), byref(f), byref(q)),
                "gcp_slice_loss")
        return f.value, q.value

    def local_loss(self, X: torch.Tensor, s_x: torch.Tensor) -> float:
        """Local reconstruction loss of a dense slice (NaN when ||X|| = 0)."""
        out = c_double(0.0)
        sl = _dense_slice(X)
        N.check(self.lib.gcp_local_loss(self.handle, byref(sl), _ptr(s_x.contiguous()), byref(out)),
                "gcp_local_loss")
        return out.value

    def ktensor_score(self, w_a: torch.Tensor, B: Sequence[torch.Tensor], w_b: torch.Tensor) -> float:
        """Congruence score of the current factors (weights w_a) against the
        reference K-tensor (B, w_b)."""
        B = [b.contiguous() for b in B]
        out = c_double(0.0)
        N.check(self.lib.gcp_ktensor_score(self.handle, _ptr(w_a.contiguous()), _ptr_array(B, 3),
                                           _ptr(w_b.contiguous()), int(B[0].shape[1]), byref(out)),
                "gcp_ktensor_score")
        return out.value

    def update_factors(self, X_t, s_t: torch.Tensor) -> None:
        sl = _slice(X_t)
        N.check(self.lib.gcp_update_factors(self.handle, byref(sl), _ptr(s_t.contiguous())),
                "gcp_update_factors")

    def step(self, X_t: torch.Tensor) -> torch.Tensor:
        """One OnlineGCP time step (Algorithm 1 body): s_t, then the factors."""
        s_t = self.solve_st(X_t)
        self.update_factors(X_t, s_t)
        return s_t

    def factors(self) -> List[torch.Tensor]:
        out = [torch.empty(n, self.rank, dtype=self.dtype, device=self.device) for n in self.dims]
        N.check(self.lib.gcp_get_factors(self.handle, _ptr_array(out, 3)), "gcp_get_factors")
        return out

    def info(self):
        t = c_int64(0)
        nw = c_int32(0)
        it = c_int64(0)
        slots = (c_int64 * max(1, self.window))()
        call = c_int64(0)
        N.check(self.lib.gcp_stream_info(self.handle, byref(t), byref(nw), byref(it), slots,
                                         byref(call)),
                "gcp_stream_info")
        return {"t": t.value, "n_window": nw.value, "adam_iter": it.value,
                "slot_times": [slots[i] for i in range(nw.value)], "sample_call": call.value}

    def kernel_timing(self, enable: bool, capacity: int = 0) -> None:
        N.check(self.lib.gcp_kernel_timing(self.handle, int(enable), int(capacity)),
                "gcp_kernel_timing")

    def kernel_time(self):
        ms = ctypes.c_double(0.0)
        n = c_int64(0)
        N.check(self.lib.gcp_kernel_time(self.handle, byref(ms), byref(n)), "gcp_kernel_time")
        return ms.value, n.value

    def autotune(self, X_t: torch.Tensor, cache_path: Optional[str] = None) -> int:
        """Times the candidate work plans and keeps the fastest (synchronous)."""
        sl = _slice(X_t)
        chosen = c_int32(0)
        N.check(self.lib.gcp_autotune(self.handle, byref(sl),
                                      cache_path.encode() if cache_path else None, byref(chosen)),
                "gcp_autotune")
        return chosen.value

    def sync(self) -> int:
        return int(self.lib.gcp_stream_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            torch.cuda.synchronize(self.device)
            self.lib.gcp_stream_destroy(self.handle)
            self.handle = c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def loss_grad_static(dims, rank: int, loss: str, X_t: torch.Tensor, A: Sequence[torch.Tensor],
                     s_t: torch.Tensor, X_hist: Optional[torch.Tensor] = None,
                     s_hist: Optional[torch.Tensor] = None, t_hist: Sequence[int] = (),
                     t: Optional[int] = None, *, w=1.0, theta=1.0, lam=0.0, mu=0.0,
                     kernel: str = "auto", want_loss: bool = True, want_grad: bool = True, out=None):
    """gcp_loss_grad_static: the dense objective and gradients with no stream
    handle or workspace (the partial sums use the library's fixed per-GPU
    array).  X_hist: contiguous [n_hist, I1, I2, I3] window slices (or None);
    t defaults to max(t_hist) + 1.  Output tensors are created unless `out`
    = (loss, [G1, G2, G3], g_s) is given, which allocates nothing."""
    lib = N.load()
    n_hist = 0 if X_hist is None else int(X_hist.shape[0])
    th = list(t_hist)
    if len(th) != n_hist:
        raise ValueError("t_hist needs one time stamp per window slice")
    if t is None:
        t = (max(th) + 1) if th else 1
    params = make_params(dims, rank, n_hist, loss, w=w, theta=theta, lam=lam, mu=mu, dtype=X_t.dtype,
                         kernel=kernel)
    dev = X_t.device
    if out is None:
        out = (torch.empty(1, dtype=X_t.dtype, device=dev),
               [torch.empty(int(n), int(rank), dtype=X_t.dtype, device=dev) for n in dims],
               torch.empty(int(rank), dtype=X_t.dtype, device=dev))
    loss_t, G, g_s = out
    sl = _dense_slice(X_t)
    want = (N.WANT_LOSS if want_loss else 0) | (N.WANT_GRAD if want_grad else 0)
    tarr = (c_int64 * max(1, n_hist))(*th)
    xh = None if X_hist is None else X_hist
    if xh is not None and not xh.is_contiguous():
        raise ValueError("X_hist must be contiguous")
    sh = None if s_hist is None else s_hist.contiguous()
    N.check(lib.gcp_loss_grad_static(byref(params), byref(sl), n_hist, _ptr(xh), _ptr(sh), tarr, int(t),
                                     _ptr_array([a.contiguous() for a in A], 3), _ptr(s_t.contiguous()), want,
                                     _ptr(loss_t), _ptr_array(G, 3), _ptr(g_s),
                                     c_void_p(torch.cuda.current_stream(dev).cuda_stream)),
            "gcp_loss_grad_static")
    return loss_t, G, g_s


# names of the C calls, for callers that want them one-to-one
def gcp_stream_init(*a, **kw) -> Stream:
    return Stream(*a, **kw)


def gcp_loss_grad(stream: Stream, X_t, A, s_t, **kw):
    return stream.loss_grad(X_t, A, s_t, **kw)


def gcp_solve_st(stream: Stream, X_t, out=None):
    return stream.solve_st(X_t, out)


def gcp_update_factors(stream: Stream, X_t, s_t):
    return stream.update_factors(X_t, s_t)


class Batch:
    """Many dense streams advanced together (persistent multi-stream launch).

    inputs: per stream a fixed X_t buffer and s_t buffer (refresh their
    contents before each call); outputs: per stream (loss, [G1, G2, G3], g_s)
    tensors written by loss_grad.  All calls run on the streams' HIP stream
    and can be captured in a torch.cuda.CUDAGraph on that stream."""

    def __init__(self, streams: Sequence[Stream], X_t: Sequence[torch.Tensor],
                 s_t: Sequence[torch.Tensor], outputs=None, autotune: bool = False,
                 tune_cache: Optional[str] = None):
        self.lib = N.load()
        self.streams = list(streams)
        n = len(self.streams)
        dev = self.streams[0].device
        self.X_t = [x.contiguous() for x in X_t]
        self.s_t = [s.contiguous() for s in s_t]
        if outputs is None:
            outputs = [(torch.empty(1, device=dev),
                        [torch.empty(d, st.rank, device=dev) for d in st.dims],
                        torch.empty(st.rank, device=dev)) for st in self.streams]
        self.outputs = outputs
        hs = (c_void_p * n)(*[st.handle.value for st in self.streams])
        io = (N.GcpBatchIO * n)()
        for i in range(n):
            io[i].X_t = self.X_t[i].data_ptr()
            io[i].s_t = self.s_t[i].data_ptr()
            loss, G, g_s = outputs[i]
            io[i].loss = loss.data_ptr()
            for k in range(3):
                io[i].G[k] = G[k].data_ptr()
            io[i].g_s = g_s.data_ptr()
        self.buckets = 0
        if autotune:
            # one tuning (or cache read) per shape bucket, before the partial
            # buffers are sized for the chosen plans
            nb = c_int32(0)
            torch.cuda.synchronize(dev)
            N.check(self.lib.gcp_batch_autotune(hs, io, n, tune_cache.encode() if tune_cache else None,
                                                byref(nb)), "gcp_batch_autotune")
            self.buckets = nb.value
        nbytes = c_size_t(0)
        N.check(self.lib.gcp_batch_workspace_size(hs, n, byref(nbytes)), "gcp_batch_workspace_size")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        handle = c_void_p(0)
        torch.cuda.synchronize(dev)
        N.check(self.lib.gcp_batch_create(hs, io, n, _ptr(self.workspace), nbytes,
                                          c_void_p(self.streams[0].hip_stream.cuda_stream),
                                          byref(handle)), "gcp_batch_create")
        self.handle = handle

    def loss_grad(self, want_loss: bool = True, want_grad: bool = True):
        want = (N.WANT_LOSS if want_loss else 0) | (N.WANT_GRAD if want_grad else 0)
        N.check(self.lib.gcp_batch_loss_grad(self.handle, want), "gcp_batch_loss_grad")
        return self.outputs

    def update_factors(self):
        N.check(self.lib.gcp_batch_update_factors(self.handle), "gcp_batch_update_factors")

    def solve_st(self):
        """Temporal weights (SGD streams, and LS for Gaussian streams) into each registered s_t."""
        N.check(self.lib.gcp_batch_solve_st(self.handle), "gcp_batch_solve_st")

    def step(self):
        """solve_st, then update_factors: one time step for every stream."""
        N.check(self.lib.gcp_batch_step(self.handle), "gcp_batch_step")

    def sync_streams(self) -> int:
        return int(self.lib.gcp_batch_sync_streams(self.handle))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.gcp_batch_destroy(self.handle)
            self.handle = c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
