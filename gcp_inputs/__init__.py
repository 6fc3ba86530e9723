"""Seeded synthetic inputs for the streaming GCP hot path.

This module is shared by the CPU oracle, the GPU tests and the bench. It
draws data only: it evaluates no loss, no derivative, no gradient and no
solve.  Planted tensors are built by multiplying out a K-tensor (sum of R
rank-one outer products, the paper's CP model of Section 2.1) purely to give
the data realistic structure; no result of either implementation depends on
that product being right, because any tensor is a valid input.

Shapes, distributions and hyperparameters follow the workloads in the
paper's Section 6 (synthetic Gaussian / Poisson experiments, Table 2) and the
five synthetic configurations this project benchmarks:

  C1  20x30x40 dense Gaussian stream, rank 4, window 3, seed 0
  C2  200^3 dense Poisson counts, rank 16, window 10, seed 1 (bench workload)
  C3  1000x1000x64 binary slices (~5% ones), rank 32, window 20, seed 2
  C4  64 independent streams, dims U{50..300}^3, rank {8,16,32}, window 4..16
  C5  2000x2000x500 sparse counts (0.1% nonzeros), rank 32, window 8, seed 4
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

LOSSES = ("gaussian", "poisson_log", "bernoulli_logit")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ktensor_full(A: List[np.ndarray], s: np.ndarray) -> np.ndarray:
    """Dense tensor of the planted K-tensor (data synthesis only)."""
    dims = tuple(a.shape[0] for a in A)
    out = np.zeros(dims, dtype=np.float64)
    for j in range(s.shape[0]):
        comp = s[j] * A[0][:, j]
        for a in A[1:]:
            comp = np.multiply.outer(comp, a[:, j])
        out += comp
    return out


@dataclass
class DenseProblem:
    """One gradient evaluation: current slice, window and evaluation point."""
    dims: tuple
    rank: int
    loss: str
    X_t: np.ndarray                 # (I1,I2,I3)
    A: List[np.ndarray]             # I_k x R
    s_t: np.ndarray                 # R
    X_hist: List[np.ndarray]        # H slices
    s_hist: np.ndarray              # H x R
    t_hist: np.ndarray              # H  (int64 time stamps)
    t: int                          # current time index
    w: float = 1.0
    theta: float = 1.0
    lam: float = 0.0
    mu: float = 0.0
    dtype: type = np.float32
    meta: dict = field(default_factory=dict)

    @property
    def window(self) -> int:
        return len(self.X_hist)

    def cast(self, dtype) -> "DenseProblem":
        """Copy with every array cast to dtype (FP32 inputs for the GPU)."""
        c = lambda a: np.ascontiguousarray(a, dtype=dtype)
        return DenseProblem(self.dims, self.rank, self.loss, c(self.X_t),
                            [c(a) for a in self.A], c(self.s_t),
                            [c(x) for x in self.X_hist],
                            c(self.s_hist.reshape(-1, self.rank)),
                            np.asarray(self.t_hist, dtype=np.int64), self.t,
                            self.w, self.theta, self.lam, self.mu, dtype,
                            dict(self.meta))

    def promoted(self) -> "DenseProblem":
        """The same values promoted exactly to FP64 (what the oracle sees)."""
        return self.cast(np.float64)


def _draw_data(g: np.random.Generator, loss: str, M: np.ndarray) -> np.ndarray:
    """Observation drawn around a planted parameter tensor M."""
    if loss == "gaussian":
        return M + g.standard_normal(M.shape)
    if loss == "poisson_log":
        return g.poisson(np.exp(np.clip(M, -20, 3))).astype(np.float64)
    if loss == "bernoulli_logit":
        p = 1.0 / (1.0 + np.exp(-M))
        return (g.random(M.shape) < p).astype(np.float64)
    if loss == "poisson_id":
        return g.poisson(np.maximum(M, 0.0)).astype(np.float64)
    if loss == "bernoulli_odds":
        M = np.maximum(M, 0.0)
        return (g.random(M.shape) < M / (1.0 + M)).astype(np.float64)
    raise ValueError(loss)


def random_dense(dims, rank: int, window: int, loss: str, seed: int,
                 w: float = 1.0, theta: float = 1.0, lam: float = 0.0,
                 mu: float = 0.0, t: Optional[int] = None,
                 dtype=np.float32) -> DenseProblem:
    """Generic parity instance: data from a random planted model, evaluated
    at an unrelated random point (so the gradient is far from stationary)."""
    g = rng(seed)
    dims = tuple(int(d) for d in dims)
    At = [g.uniform(-0.8, 0.8, size=(n, rank)) for n in dims]
    ns = window + 1
    S_true = g.uniform(0.5, 1.5, size=(ns, rank))
    Xs = [_draw_data(g, loss, ktensor_full(At, S_true[h])) for h in range(ns)]
    A = [g.uniform(-0.6, 0.6, size=(n, rank)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(ns, rank))
    if t is None:
        t = window + 1
    t_hist = np.arange(t - window, t, dtype=np.int64)
    p = DenseProblem(dims, rank, loss, Xs[-1], A, S[-1], Xs[:-1],
                     S[:-1].reshape(window, rank), t_hist, t, w, theta, lam,
                     mu, np.float64)
    return p.cast(dtype)


def weight_problem(dims, rank: int, loss: str, seed: int, dtype=np.float32):
    """Temporal-weight instance: planted factors A ~ U(-0.8, 0.8), weights
    s* ~ U(1, 3), and X_t drawn around the model [[A; s*]].  Returns
    (X_t, A, s*) with X_t and A in dtype."""
    g = rng(seed)
    dims = tuple(int(d) for d in dims)
    A = [g.uniform(-0.8, 0.8, size=(n, rank)) for n in dims]
    s_true = g.uniform(1.0, 3.0, size=rank)
    X = _draw_data(g, loss, ktensor_full(A, s_true))
    return X.astype(dtype), [a.astype(dtype) for a in A], s_true


def nonneg_dense(dims, rank: int, window: int, loss: str, seed: int, w: float = 1.0, theta: float = 1.0,
                 lam: float = 0.0, mu: float = 0.0, dtype=np.float32) -> DenseProblem:
    """Instance for the identity- and odds-link losses (m >= 0): planted
    factors U(0.1, 1), weights U(0.5, 1.5), data drawn around the planted
    model; evaluation point factors U(0.1, 1) and weights U(0.5, 1.5)."""
    g = rng(seed)
    dims = tuple(int(d) for d in dims)
    At = [g.uniform(0.1, 1.0, size=(n, rank)) for n in dims]
    ns = window + 1
    S_true = g.uniform(0.5, 1.5, size=(ns, rank))
    Xs = [_draw_data(g, loss, ktensor_full(At, S_true[h])) for h in range(ns)]
    A = [g.uniform(0.1, 1.0, size=(n, rank)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(ns, rank))
    t = window + 1
    t_hist = np.arange(1, t, dtype=np.int64)
    p = DenseProblem(dims, rank, loss, Xs[-1], A, S[-1], Xs[:-1], S[:-1].reshape(window, rank), t_hist, t, w,
                     theta, lam, mu, np.float64)
    return p.cast(dtype)


# ---------------------------------------------------------------- C1 ----
@dataclass
class PlantedStream:
    """A stream of slices drawn around a planted K-tensor (A_true, S_true[t])."""
    A_true: List[np.ndarray]
    S_true: np.ndarray   # T x R
    X: np.ndarray        # T x I1 x I2 x I3 (FP64)


def c1_stream(seed: int = 0, dims=(20, 30, 40), rank: int = 4, steps: int = 20,
              noise: float = 0.1) -> PlantedStream:
    """C1: factors N(0,1), temporal weights U(0.5,1.5), X_t = M_t plus noise
    scaled so that ||noise||_F = noise * ||M_t||_F (10% relative noise)."""
    g = rng(seed)
    A = [g.standard_normal((n, rank)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(steps, rank))
    X = np.empty((steps,) + tuple(dims))
    for t in range(steps):
        M = ktensor_full(A, S[t])
        N = g.standard_normal(M.shape)
        X[t] = M + noise * (np.linalg.norm(M) / np.linalg.norm(N)) * N
    return PlantedStream(A, S, X)


def poisson_log_stream(seed: int = 21, dims=(15, 18, 20), rank: int = 3, steps: int = 14,
                       scale: float = 0.7) -> PlantedStream:
    """Small planted count stream for the log link: factors N(0, scale^2),
    weights U(0.5,1.5), X_t ~ Poisson(exp(M_t)) where M_t is the planted
    K-tensor (the log-rate model the Poisson-log loss fits)."""
    g = rng(seed)
    A = [g.standard_normal((n, rank)) * scale for n in dims]
    S = g.uniform(0.5, 1.5, size=(steps, rank))
    X = np.stack([g.poisson(np.exp(ktensor_full(A, S[t]))).astype(np.float64) for t in range(steps)])
    return PlantedStream(A, S, X)


def c1_problem(seed: int = 0, window: int = 3, dtype=np.float32) -> DenseProblem:
    """C1 evaluation point at t = window+1: perturbed planted factors."""
    st = c1_stream(seed)
    g = rng(seed + 1000)
    A0 = [a + 0.1 * g.standard_normal(a.shape) for a in st.A_true]
    S0 = st.S_true + 0.05 * g.standard_normal(st.S_true.shape)
    t = window + 1
    p = DenseProblem(st.X.shape[1:], st.S_true.shape[1], "gaussian",
                     st.X[t - 1], A0, S0[t - 1],
                     [st.X[h - 1] for h in range(1, t)], S0[:t - 1],
                     np.arange(1, t, dtype=np.int64), t, 1.0, 1.0, 0.0, 0.0,
                     np.float64, {"config": "C1"})
    return p.cast(dtype)


# ---------------------------------------------------------------- C2 ----
def c2_planted(seed: int = 1, dims=(200, 200, 200), rank: int = 16,
               zero_frac: float = 0.7):
    """Planted nonnegative factors U(0,1) with round(0.7 I_k) rows of every
    column set to zero (chosen without replacement)."""
    g = rng(seed)
    A = []
    for n in dims:
        a = g.uniform(0.0, 1.0, size=(n, rank))
        nz = int(round(zero_frac * n))
        for j in range(rank):
            a[g.choice(n, size=nz, replace=False), j] = 0.0
        A.append(a)
    return g, A


def c2_problem(seed: int = 1, dims=(200, 200, 200), rank: int = 16,
               window: int = 10, dtype=np.float32) -> DenseProblem:
    """C2: Poisson counts X_h ~ Poisson(M_h) of a planted nonnegative model
    (identity-scale rates); log-link evaluation point A ~ U(-0.5,0.5),
    s ~ U(0.5,1.5)."""
    g, At = c2_planted(seed, dims, rank)
    ns = window + 1
    S_true = g.uniform(0.5, 1.5, size=(ns, rank))
    Xs = [g.poisson(ktensor_full(At, S_true[h])).astype(np.float64)
          for h in range(ns)]
    A = [g.uniform(-0.5, 0.5, size=(n, rank)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(ns, rank))
    t = window + 1
    p = DenseProblem(tuple(dims), rank, "poisson_log", Xs[-1], A, S[-1],
                     Xs[:-1], S[:-1], np.arange(1, t, dtype=np.int64), t,
                     meta={"config": "C2"}, dtype=np.float64)
    return p.cast(dtype)


# ---------------------------------------------------------------- C3 ----
def c3_planted(seed: int = 2, dims=(1000, 1000, 64), rank: int = 32,
               target: float = 0.05, sample: int = 1_000_000):
    """Planted rank-R logit: column 0 is an all-ones bias of weight beta, the
    other columns N(0, 0.56^2) with weights U(0.5,1.5).  beta is set by
    bisection so that the mean of sigmoid(M) over a random sample is
    `target` (about 5% ones)."""
    g = rng(seed)
    A = [g.normal(0.0, 0.56, size=(n, rank)) for n in dims]
    for a in A:
        a[:, 0] = 1.0
    s = g.uniform(0.5, 1.5, size=rank)
    idx = [g.integers(0, n, size=sample) for n in dims]
    rest = np.zeros(sample)
    for j in range(1, rank):
        rest += s[j] * A[0][idx[0], j] * A[1][idx[1], j] * A[2][idx[2], j]
    lo, hi = -20.0, 5.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if np.mean(1.0 / (1.0 + np.exp(-(rest + mid)))) > target:
            hi = mid
        else:
            lo = mid
    s = s.copy()
    s[0] = 0.5 * (lo + hi)
    return g, A, s


def c3_problem(seed: int = 2, dims=(1000, 1000, 64), rank: int = 32,
               window: int = 20, dtype=np.float32) -> DenseProblem:
    """C3 structure at any dims (full size is generated on the device by the
    bench; small dims serve the FP64 gradcheck sub-instance 16x16x8)."""
    g, At, s_pl = c3_planted(seed, dims, rank,
                             sample=min(1_000_000, int(np.prod(dims))))
    ns = window + 1
    Xs = []
    for h in range(ns):
        sh = s_pl.copy()
        sh[1:] *= g.uniform(0.8, 1.2, size=rank - 1)
        M = ktensor_full(At, sh)
        Xs.append((g.random(M.shape) < 1.0 / (1.0 + np.exp(-M))).astype(np.float64))
    A = [a + 0.05 * g.standard_normal(a.shape) for a in At]
    S = np.stack([s_pl * g.uniform(0.9, 1.1, size=rank) for _ in range(ns)])
    t = window + 1
    p = DenseProblem(tuple(dims), rank, "bernoulli_logit", Xs[-1], A, S[-1],
                     Xs[:-1], S[:-1], np.arange(1, t, dtype=np.int64), t,
                     meta={"config": "C3"}, dtype=np.float64)
    return p.cast(dtype)


# ---------------------------------------------------------------- C4 ----
@dataclass
class StreamSpec:
    dims: tuple
    rank: int
    window: int
    loss: str
    seed: int


def c4_specs(seed: int = 3, n_streams: int = 64, lo: int = 50, hi: int = 300):
    """C4: per stream dims ~ U{50..300}^3, rank ~ U{8,16,32}, window ~
    U{4..16}; Gaussian for even stream index, Poisson-log for odd."""
    g = rng(seed)
    specs = []
    for i in range(n_streams):
        dims = tuple(int(v) for v in g.integers(lo, hi + 1, size=3))
        rank = int(g.choice([8, 16, 32]))
        window = int(g.integers(4, 17))
        loss = "gaussian" if i % 2 == 0 else "poisson_log"
        specs.append(StreamSpec(dims, rank, window, loss, seed * 1000 + i))
    return specs


# ---------------------------------------------------------------- C5 ----
@dataclass
class CooSlice:
    dims: tuple
    coords: np.ndarray   # nnz x 3 int32, sorted by row-major linear index
    vals: np.ndarray     # nnz float


def random_coo(g: np.random.Generator, dims, nnz: int) -> CooSlice:
    """nnz distinct uniform linear indices (draw, sort-unique, top up), values
    Poisson(3)+1, sorted by row-major linear index."""
    omega = int(np.prod(dims))
    lin = np.unique(g.integers(0, omega, size=nnz))
    while lin.size < nnz:
        extra = g.integers(0, omega, size=nnz - lin.size)
        lin = np.unique(np.concatenate([lin, extra]))
    coords = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int32)
    vals = (g.poisson(3.0, size=nnz) + 1).astype(np.float64)
    return CooSlice(tuple(dims), coords, vals)


@dataclass
class SparseProblem:
    dims: tuple
    rank: int
    X_t: CooSlice
    A: List[np.ndarray]
    s_t: np.ndarray
    X_hist: List[CooSlice]
    s_hist: np.ndarray
    t_hist: np.ndarray
    t: int
    p: int
    q: int
    seed: int
    iteration: int = 0
    w: float = 1.0
    theta: float = 1.0
    lam: float = 0.0
    mu: float = 0.0
    loss: str = "poisson_log"


def sparse_problem(dims=(2000, 2000, 500), rank: int = 32, window: int = 8,
                   nnz: int = 2_000_000, p: Optional[int] = None,
                   q: Optional[int] = None, seed: int = 4,
                   loss: str = "poisson_log") -> SparseProblem:
    """C5 structure at any dims: COO slices, factors U(-0.5,0.5), weights
    U(0.5,1.5); p = q = nnz by default."""
    g = rng(seed)
    ns = window + 1
    slices = [random_coo(g, dims, nnz) for _ in range(ns)]
    if loss == "bernoulli_logit":
        for sl in slices:
            sl.vals[:] = 1.0
    A = [g.uniform(-0.5, 0.5, size=(n, rank)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(ns, rank))
    t = window + 1
    return SparseProblem(tuple(dims), rank, slices[-1], A, S[-1], slices[:-1],
                         S[:-1], np.arange(1, t, dtype=np.int64), t,
                         nnz if p is None else p, nnz if q is None else q,
                         seed, 0, loss=loss)


# ------------------------------------------------- on-device synthesis --
def device_dense_window(dims, rank: int, window: int, loss: str, seed: int, device="cuda"):
    """Random full-size inputs on the device for timing (torch generator):
    slices drawn from the loss's distribution around a random planted
    parameter of the given rank, evaluation point factors U(-0.5, 0.5)
    (Poisson) or N(0, 0.3^2) (others), weights U(0.5, 1.5)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    ns = window + 1

    def planted(scale):
        A = [torch.rand(n, rank, generator=g, device=device) * 2 - 1 for n in dims]
        s = torch.rand(rank, generator=g, device=device) + 0.5
        M = torch.einsum("ir,jr,kr->ijk", (A[0] * s * scale).contiguous(), A[1].contiguous(),
                         A[2].contiguous())
        return M

    Xs = []
    for _ in range(ns):
        M = planted(0.3)
        if loss == "gaussian":
            X = M + torch.randn(M.shape, generator=g, device=device)
        elif loss == "poisson_log":
            X = torch.poisson(torch.exp(M.clamp(max=3.0)), generator=g)
        else:
            X = (torch.rand(M.shape, generator=g, device=device) < torch.sigmoid(M - 3.0)).float()
        Xs.append(X.contiguous())
        del M
    A = [(torch.rand(n, rank, generator=g, device=device) - 0.5).contiguous() for n in dims]
    S = torch.rand(ns, rank, generator=g, device=device) + 0.5
    return Xs[-1], A, S[-1].contiguous(), Xs[:-1], S[:-1].contiguous()


def pack_bits(x: np.ndarray) -> np.ndarray:
    """Bit-packed storage of a binary slice (any shape, last axis I3): every
    row of I3 entries becomes ceil(I3/32) uint32 words, entry i3 in bit
    i3 % 32 of word i3 // 32 (least significant bit first), padding bits 0.
    Non-zero entries are ones."""
    x = np.asarray(x)
    I3 = x.shape[-1]
    nw = (I3 + 31) // 32
    padded = np.zeros(x.shape[:-1] + (nw * 32,), np.uint8)
    padded[..., :I3] = x != 0
    b = np.packbits(padded, axis=-1, bitorder="little")
    return np.ascontiguousarray(b).view("<u4").reshape(x.shape[:-1] + (nw,))


def device_pack_bits(x):
    """pack_bits of a device tensor, as int32 words (the same bits)."""
    import torch
    I3 = x.shape[-1]
    nw = (I3 + 31) // 32
    xb = torch.zeros(x.shape[:-1] + (nw * 32,), dtype=torch.int64, device=x.device)
    xb[..., :I3] = (x != 0).to(torch.int64)
    w = (xb.view(*x.shape[:-1], nw, 32) << torch.arange(32, device=x.device)).sum(-1)
    w = torch.where(w >= 2 ** 31, w - 2 ** 32, w)
    return w.to(torch.int32).contiguous()
