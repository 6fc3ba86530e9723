"""Matrix slices (d = 2): a stream of I1 x I2 slices with model
m_ij = sum_r s_r a_ir b_jr, against the oracle's two-way reading (I3 = 1
and a fixed row of ones, pinned against the two-way formulas)."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import sampled as osm
from oracle.stream import StreamOracle

from helpers import TOL, loss_err, grad_err, rel_err

pytestmark = pytest.mark.gpu


def _data(g, loss, shape):
    if loss == "gaussian":
        return g.normal(size=shape)
    if loss == "poisson_log":
        return g.poisson(1.0, size=shape).astype(float)
    return (g.random(shape) < 0.3).astype(float)


def _case(loss, dims, R, H, seed, dtype):
    g = np.random.default_rng(seed)
    A = [g.uniform(-0.6, 0.6, (n, R)) for n in dims]
    Xh = [_data(g, loss, dims) for _ in range(H)]
    Sh = g.uniform(0.5, 1.5, (H, R))
    X = _data(g, loss, dims)
    s = g.uniform(0.5, 1.5, R)
    return A, Xh, Sh, X, s


def _stream(loss, dims, R, A, Xh, Sh, dtype, **kw):
    import torch
    from paper_2110_14514_amd import Stream
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)
    H = len(Xh)
    st = Stream(dims, R, H, loss, [T(a) for a in A], [T(x) for x in Xh], T(Sh) if H else None,
                list(range(1, H + 1)), **kw)
    return st, T


@pytest.mark.parametrize("loss", og.LOSSES)
@pytest.mark.parametrize("kernel,dtype_name", [("valu", "float32"), ("mfma", "float32"), ("auto", "float64")])
@pytest.mark.parametrize("dims,R,H", [((30, 40), 8, 3), ((300, 300), 20, 5), ((17, 9), 16, 0)])
def test_loss_grad_matches_two_way_oracle(dims, R, H, kernel, dtype_name, loss):
    import torch
    print("case: d2 loss_grad", dims, R, H, kernel, dtype_name, loss, flush=True)
    dtype = getattr(torch, dtype_name)
    A, Xh, Sh, X, s = _case(loss, dims, R, H, seed=R + H, dtype=dtype)
    kw = dict(w=1.2, theta=0.9, lam=0.05, mu=0.2)
    st, T = _stream(loss, dims, R, A, Xh, Sh, dtype, kernel=kernel, **kw)
    if dtype == torch.float32:   # the oracle sees the FP32 inputs
        A = [a.astype(np.float32).astype(np.float64) for a in A]
        Xh = [x.astype(np.float32).astype(np.float64) for x in Xh]
        Sh, X, s = (v.astype(np.float32).astype(np.float64) for v in (Sh, X, s))
    loss_v, G, gs = st.loss_grad(T(X), [T(a) for a in A], T(s))
    torch.cuda.synchronize()
    assert st.sync() == 0 and len(G) == 2
    orc = StreamOracle(A, Xh, Sh, list(range(1, H + 1)), loss=loss, window=H, d=2, **kw)
    F = orc.factor_objective(X, s) + 0.5 * kw["mu"] * float(s @ s)
    Gr, gsr = og.gradient(orc.problem(X.reshape(dims + (1,)), s))
    tol = TOL if dtype == torch.float32 else 1e-12
    scale = og.loss_terms_abs(orc.problem(X.reshape(dims + (1,)), s))
    assert loss_err(loss_v.item(), F, scale) <= tol
    for k in range(2):
        assert grad_err(G[k].double().cpu().numpy(), Gr[k]) <= tol, k
    assert grad_err(gs.double().cpu().numpy(), gsr) <= tol


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log"])
def test_stream_steps_with_both_sgd_solvers(loss):
    """Three OnlineGCP steps on matrix slices: Algorithm 3 (or the LS solve
    for Gaussian) and Algorithm 4 epochs, factors and weights in FP64."""
    import torch
    print("case: d2 steps", loss, flush=True)
    dims, R, H = (40, 30), 5, 3
    A, Xh, Sh, X, s = _case(loss, dims, R, H, seed=7, dtype=torch.float64)
    kw = dict(w=1.1, theta=0.9, lam=0.05, mu=0.1, tau_f=3, kappa_f=3, alpha_f=0.05, seed=2)
    if loss != "gaussian":
        kw.update(tsolve="sgd", tau_w=4, kappa_w=3, alpha_w=0.05)
    st, T = _stream(loss, dims, R, A, Xh, Sh, torch.float64, **kw)
    orc = StreamOracle(A, Xh, Sh, list(range(1, H + 1)), loss=loss, window=H, d=2, **kw)
    g = np.random.default_rng(11)
    for step in range(3):
        Xn = _data(g, loss, dims)
        sv = st.step(T(Xn))
        sr = orc.step(Xn)
        assert st.sync() == 0
        assert st.factor_info()["rolled"] == orc.fac_info.rolled
        assert rel_err(sv.cpu().numpy(), sr) <= 1e-9
        F = st.factors()
        assert len(F) == 2
        for k in range(2):
            assert rel_err(F[k].cpu().numpy(), orc.A[k]) <= 1e-9, (step, k)


def test_sampled_matrix_slices_match_oracle():
    """COO matrix slices (coords (i1, 0, i2): the stream's I1 x 1 x I2
    layout): the sampled objective and gradients of the two free factors."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: d2 sampled", flush=True)
    prob = gi.sparse_problem(dims=(60, 1, 50), rank=6, window=2, nnz=600, p=800, q=800, seed=3, loss="poisson_log")
    R = 6
    prob.A = [prob.A[0].astype(np.float32).astype(np.float64), np.ones((1, R)),
              prob.A[2].astype(np.float32).astype(np.float64)]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    prob.s_hist = prob.s_hist.astype(np.float32).astype(np.float64)
    for sl in [prob.X_t] + list(prob.X_hist):
        sl.vals = sl.vals.astype(np.float32).astype(np.float64)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    C = lambda sl: (torch.from_numpy(np.ascontiguousarray(sl.coords, dtype=np.int32)).cuda(), T(sl.vals))
    st = Stream((60, 50), R, 2, "poisson_log", [T(prob.A[0]), T(prob.A[2])], [C(x) for x in prob.X_hist],
                T(prob.s_hist), list(prob.t_hist), w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu,
                seed=prob.seed, slice_kind="coo", max_nnz=600, p=800, q=800)
    loss_v, G, gs = st.loss_grad(C(prob.X_t), [T(prob.A[0]), T(prob.A[2])], T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    F, Gr, gsr = osm.sampled_loss_grad(prob, call=0)
    F -= 0.5 * prob.lam * R          # the fixed row is not regularised
    assert loss_err(loss_v.item(), F, abs(F)) <= TOL
    for k, ko in ((0, 0), (1, 2)):
        assert grad_err(G[k].double().cpu().numpy(), Gr[ko]) <= TOL
    assert grad_err(gs.double().cpu().numpy(), gsr) <= TOL


def test_matrix_slice_metrics_and_score():
    """Slice loss and K-tensor score take the caller's two factors."""
    import torch
    from oracle import metrics as om
    print("case: d2 metrics", flush=True)
    g = np.random.default_rng(21)
    dims, R = (40, 30), 5
    A = [g.uniform(-0.6, 0.6, (n, R)) for n in dims]
    X = g.normal(size=dims)
    s = g.uniform(0.5, 1.5, R)
    st, T = _stream("gaussian", dims, R, A, [], np.zeros((0, R)), torch.float64)
    f, q = st.slice_loss(T(X), T(s))
    M = A[0] @ np.diag(s) @ A[1].T
    assert f == pytest.approx(float(np.sum((X - M) ** 2)), rel=1e-12) and q == pytest.approx(float(np.sum(X * X)))
    B = [a[:, ::-1] * 2.0 for a in A]
    score = st.ktensor_score(T(s), [T(b) for b in B], T(s[::-1] / 4.0))
    assert score == pytest.approx(om.ktensor_score(A, s, B, s[::-1] / 4.0), rel=1e-12)
