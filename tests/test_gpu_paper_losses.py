"""The identity-link Poisson and odds-link Bernoulli losses of Section 2.2
(m >= 0, log(m + 1e-10)) through every kernel family: fused dense (vector
and matrix-core), FP64, unfused, sampled COO, and both SGD solvers."""
from types import SimpleNamespace

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import sampled as osm
from oracle import temporal_sgd as ots
from oracle.stream import StreamOracle

from helpers import TOL, compare, gpu_loss_grad, loss_err, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [((5, 6, 7), 4, 0), ((7, 9, 70), 5, 2), ((17, 33, 129), 16, 3), ((9, 4, 64), 32, 1),
          ((6, 5, 200), 16, 20), ((11, 13, 52), 16, 6)]


@pytest.mark.parametrize("kernel", ["valu", "mfma"])
@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
@pytest.mark.parametrize("dims,R,H", SHAPES)
def test_fused_matches_oracle(dims, R, H, loss, kernel):
    print("case: fused", kernel, dims, R, H, loss, flush=True)
    prob = gi.nonneg_dense(dims, R, H, loss, seed=R + H, w=1.3, theta=0.8, lam=0.05, mu=0.2)
    got, code, _ = gpu_loss_grad(prob, kernel=kernel)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_fp64_and_plain_match_oracle(loss):
    print("case: fp64/plain", loss, flush=True)
    p64 = gi.nonneg_dense((7, 9, 70), 6, 3, loss, seed=2, lam=0.1, mu=0.1, dtype=np.float64)
    got, code, _ = gpu_loss_grad(p64)
    assert code == 0 and max(compare(p64, got, og).values()) <= 1e-12
    p32 = gi.nonneg_dense((20, 30, 40), 8, 4, loss, seed=3, lam=0.1, mu=0.1)
    got, code, _ = gpu_loss_grad(p32, plain=True)
    assert code == 0 and max(compare(p32, got, og).values()) <= TOL


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_sampled_gradient_matches_oracle(loss):
    """COO slices with nonnegative factors and weights: the sampled
    objective and gradient equal the oracle's over the same draws."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: sampled", loss, flush=True)
    prob = gi.sparse_problem(dims=(25, 30, 35), rank=8, window=2, nnz=1200, p=1500, q=1500, seed=5, loss=loss)
    prob.A = [(np.abs(a) + 0.05).astype(np.float32).astype(np.float64) for a in prob.A]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    prob.s_hist = prob.s_hist.astype(np.float32).astype(np.float64)
    for sl in [prob.X_t] + list(prob.X_hist):
        if loss == "bernoulli_odds":
            sl.vals[:] = 1.0
        sl.vals = sl.vals.astype(np.float32).astype(np.float64)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    C = lambda sl: (torch.from_numpy(np.ascontiguousarray(sl.coords, dtype=np.int32)).cuda(), T(sl.vals))
    st = Stream(prob.dims, 8, 2, loss, [T(a) for a in prob.A], [C(x) for x in prob.X_hist], T(prob.s_hist),
                list(prob.t_hist), w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu, seed=prob.seed,
                slice_kind="coo", max_nnz=1200, p=1500, q=1500)
    loss_v, G, gs = st.loss_grad(C(prob.X_t), [T(a) for a in prob.A], T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    F, Gr, gsr = osm.sampled_loss_grad(prob, call=0)
    assert loss_err(loss_v.item(), F, abs(F)) <= TOL
    for k in range(3):
        assert rel_err(G[k].double().cpu().numpy(), Gr[k]) <= TOL
    assert rel_err(gs.double().cpu().numpy(), gsr) <= TOL


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_weight_sgd_matches_oracle(loss):
    """Algorithm 3 with the bound l = 0 (the losses need m >= 0)."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: weight sgd", loss, flush=True)
    p = gi.nonneg_dense((9, 7, 150), 5, 0, loss, seed=4, dtype=np.float64)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(p.dims, 5, 0, loss, [T(a) for a in p.A], tsolve="sgd", tau_w=6, kappa_w=4, alpha_w=0.1,
                lower=0.0, mu=0.1)
    s = st.solve_st(T(p.X_t)).cpu().numpy()
    info = st.solve_info()
    assert st.sync() == 0
    ref, rinfo = ots.temporal_sgd(p.X_t, p.A, loss, mu=0.1, lower=0.0, alpha=0.1, tau=6, kappa=4)
    assert all(abs(t - f) > 1e-10 * abs(f) for t, f in zip(rinfo.F_try, rinfo.F[:-1]))
    assert info["rolled"] == rinfo.rolled and np.all(s >= 0)
    assert rel_err(s, ref) <= 1e-9


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_online_steps_with_factor_epochs(loss):
    """Two OnlineGCP steps (Algorithm 3 + Algorithm 4 epochs, l = 0) in FP64."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: online steps", loss, flush=True)
    p = gi.nonneg_dense((10, 8, 50), 4, 2, loss, seed=6, dtype=np.float64)
    kw = dict(w=1.1, theta=0.9, lam=0.05, mu=0.1, tau_f=3, kappa_f=3, alpha_f=0.05, lower=0.0, seed=2,
              tsolve="sgd", tau_w=4, kappa_w=3, alpha_w=0.05)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(p.dims, 4, 2, loss, [T(a) for a in p.A], [T(x) for x in p.X_hist], T(p.s_hist),
                [int(t) for t in p.t_hist], **kw)
    orc = StreamOracle(p.A, p.X_hist, p.s_hist, p.t_hist, loss=loss, window=2, **kw)
    g = np.random.default_rng(9)
    for step in range(2):
        X = gi._draw_data(g, loss, gi.ktensor_full([np.abs(a) for a in p.A], np.ones(4)))
        s = st.step(T(X))
        s_ref = orc.step(X)
        assert st.sync() == 0
        assert st.solve_info()["rolled"] == orc.solve_info.rolled
        assert st.factor_info()["rolled"] == orc.fac_info.rolled
        assert rel_err(s.cpu().numpy(), s_ref) <= 1e-9
        for k, a in enumerate(st.factors()):
            assert rel_err(a.cpu().numpy(), orc.A[k]) <= 1e-9, (step, k)
