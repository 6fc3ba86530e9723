"""Windows above 64 slots with the model-difference history (the paper's
window of 500 for its crime-count stream, Section 6.2): the window keeps R
weights and a time stamp per slot, the weights w_h = w theta^(t - t_h) are
formed on the device from device-held stamps, and the history term sums
all slots in FP64."""
from types import SimpleNamespace

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import model_hist as mh
from oracle import sampled as osm
from oracle.stream import StreamOracle

from helpers import TOL, grad_err, loss_err, rel_err

pytestmark = pytest.mark.gpu


def _case(dims, R, H, loss, seed, dtype):
    prob = gi.random_dense(dims, R, H, loss, seed=seed, w=1.1, theta=0.995, lam=0.05, mu=0.1, dtype=dtype)
    g = np.random.default_rng(seed + 1000)
    A_old = [(a + 0.05 * g.uniform(-1, 1, size=a.shape)).astype(dtype) for a in prob.A]
    return prob, A_old


@pytest.mark.parametrize("H,dtype", [(65, np.float32), (500, np.float32), (500, np.float64), (2000, np.float64)])
def test_long_model_window_matches_oracle(H, dtype):
    import torch
    from paper_2110_14514_amd import Stream
    print("case: long model window", H, dtype.__name__, flush=True)
    prob, A_old = _case((12, 10, 30), 8, H, "poisson_log", seed=H, dtype=dtype)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(prob.dims, prob.rank, H, prob.loss, [T(a) for a in A_old], [],
                T(np.asarray(prob.s_hist).reshape(H, prob.rank)), list(prob.t_hist), w=prob.w,
                theta=prob.theta, lam=prob.lam, mu=prob.mu, hist="model")
    lv, G, gs = st.loss_grad(T(prob.X_t), [T(a) for a in prob.A], T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    f64 = lambda a: np.asarray(a, np.float64)
    p = SimpleNamespace(X_t=f64(prob.X_t), A=[f64(a) for a in prob.A], A_old=[f64(a) for a in A_old],
                        s_t=f64(prob.s_t), s_hist=f64(prob.s_hist), t_hist=np.asarray(prob.t_hist), t=prob.t,
                        w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu, loss=prob.loss)
    F = mh.objective_model(p)
    Gr, gsr = mh.gradient_model(p)
    c = og.history_weights(p.t, p.t_hist, p.w, p.theta)
    scale = og.loss_terms_abs(mh._current_only(p)) + mh.history_objective(p.A, p.A_old, p.s_hist, c)
    tol = TOL if dtype == np.float32 else 1e-11
    assert loss_err(lv.item(), F, scale) <= tol
    for k in range(3):
        assert grad_err(G[k].double().cpu().numpy(), Gr[k]) <= tol, k
    assert grad_err(gs.double().cpu().numpy(), gsr) <= tol


def test_long_model_window_steps_match_oracle():
    """A window of 300 slots that starts with 298: two appends, then the
    reservoir draws (slot choice, stamps and weights) against the oracle,
    FP64, with LS weights and factor epochs."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: long model window steps", flush=True)
    H, n0, dims, R = 300, 298, (9, 8, 10), 4
    g = np.random.default_rng(5)
    A0 = [g.uniform(-0.6, 0.6, (n, R)) for n in dims]
    S0 = g.uniform(0.5, 1.5, (n0, R))
    kw = dict(w=1.0, theta=0.99, lam=0.01, mu=0.02, alpha_f=1e-2, tau_f=2, kappa_f=2, seed=13)
    orc = StreamOracle(A0, [], S0, np.arange(1, n0 + 1), loss="gaussian", window=H, hist="model", **kw)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(dims, R, H, "gaussian", [T(a) for a in A0], [], T(S0), list(range(1, n0 + 1)), hist="model", **kw)
    for step in range(6):
        X = g.normal(size=dims)
        sv = st.step(T(X))
        sr = orc.step(X)
        assert st.sync() == 0
        assert rel_err(sv.cpu().numpy(), sr) <= 1e-9, step
        info = st.info()
        assert info["t"] == orc.t and info["slot_times"] == orc.slots, step
        for a, b in zip(st.factors(), orc.A):
            assert rel_err(a.cpu().numpy(), b) <= 1e-9, step
    assert len(orc.slots) == H


def test_long_model_window_coo():
    """COO slices with a model-difference window of 200 slots."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: long model window coo", flush=True)
    prob = gi.sparse_problem(dims=(30, 40, 50), rank=8, window=2, nnz=2000, p=3000, q=3000, seed=9,
                             loss="poisson_log")
    H = 200
    g = np.random.default_rng(10)
    prob.A = [a.astype(np.float32).astype(np.float64) for a in prob.A]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    prob.X_t.vals = prob.X_t.vals.astype(np.float32).astype(np.float64)
    prob.s_hist = g.uniform(0.5, 1.5, (H, 8)).astype(np.float32).astype(np.float64)
    prob.t_hist = np.arange(1, H + 1)
    prob.t = H + 1
    prob.lam, prob.mu, prob.theta, prob.w = 0.05, 0.1, 0.99, 1.3
    A_old = [(a + 0.05 * g.uniform(-1, 1, size=a.shape)).astype(np.float32).astype(np.float64) for a in prob.A]
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    coo = lambda sl: (torch.from_numpy(np.ascontiguousarray(sl.coords, dtype=np.int32)).cuda(), T(sl.vals))
    st = Stream(prob.dims, prob.rank, H, prob.loss, [T(a) for a in A_old], [], T(prob.s_hist), list(prob.t_hist),
                w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu, seed=prob.seed, slice_kind="coo",
                max_nnz=prob.X_t.coords.shape[0], p=prob.p, q=prob.q, hist="model")
    lv, G, gs = st.loss_grad(coo(prob.X_t), [T(a) for a in prob.A], T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    cur = SimpleNamespace(**vars(prob))
    cur.X_hist = []
    cur.s_hist = np.zeros((0, 8))
    cur.t_hist = np.zeros(0, np.int64)
    F, Gr, gsr = osm.sampled_loss_grad(cur, call=0)
    c = og.history_weights(prob.t, prob.t_hist, prob.w, prob.theta)
    F += mh.history_objective(prob.A, A_old, prob.s_hist, c)
    Gh = mh.history_gradient(prob.A, A_old, prob.s_hist, c)
    assert loss_err(lv.item(), F, max(abs(F), 1.0)) <= TOL
    for k in range(3):
        assert grad_err(G[k].double().cpu().numpy(), Gr[k] + Gh[k]) <= TOL, k
    assert grad_err(gs.double().cpu().numpy(), gsr) <= TOL
