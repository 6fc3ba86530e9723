"""Device-side epochs of the factor solver (Algorithm 4 with the ADAM Update
of Algorithm 2) against the FP64 oracle stream: factors, decisions, rate and
iteration index over several time steps; stopping test; both histories; a
full OnlineGCP step with both SGD solvers."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle.stream import StreamOracle

from helpers import rel_err

pytestmark = pytest.mark.gpu

KW = dict(w=1.1, theta=0.9, lam=0.05, mu=0.3, tau_f=3, seed=2, kappa_f=4)


def _pair(prob, dtype, hist="slices", **kw):
    import torch
    from paper_2110_14514_amd import Stream
    opts = dict(KW)
    opts.update(kw)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)
    H = len(prob.t_hist)
    Xh = [T(x) for x in prob.X_hist] if hist == "slices" else []
    st = Stream(prob.dims, prob.rank, H, prob.loss, [T(a) for a in prob.A], Xh, T(prob.s_hist),
                [int(t) for t in prob.t_hist], hist=hist, **opts)
    orc = StreamOracle(prob.A, prob.X_hist if hist == "slices" else [], prob.s_hist, prob.t_hist, loss=prob.loss,
                       window=H, hist=hist, **opts)
    return st, orc, T


def _clear(info, margin):
    return all(abs(t - f) > margin * abs(f) for t, f in zip(info.F_try, info.F[:-1]))


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_epochs_match_oracle_over_steps(loss, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    print("case: epochs", loss, dtype_name, flush=True)
    prob = gi.random_dense((9, 7, 40), 5, 3, loss, 3, dtype=np.float64)
    st, orc, T = _pair(prob, dtype, alpha_f=1.0)
    fp64 = dtype == torch.float64
    for step in range(3):
        st.update_factors(T(prob.X_t), T(prob.s_t))
        orc.update_factors(prob.X_t, prob.s_t)
        info = st.factor_info()
        assert st.sync() == 0
        assert _clear(orc.fac_info, 1e-10 if fp64 else 1e-4)
        assert info["rolled"] == orc.fac_info.rolled, step
        assert info["iters"] == orc.i and st.info()["adam_iter"] == orc.i
        assert info["alpha"] == pytest.approx(orc.alpha_f, rel=1e-15)
        assert abs(info["F"] - orc.fac_info.F[-1]) <= (1e-11 if fp64 else 1e-5) * abs(orc.fac_info.F[-1])
        for k, a in enumerate(st.factors()):
            assert rel_err(a.double().cpu().numpy(), orc.A[k]) <= (1e-9 if fp64 else 1e-4), (step, k)


def test_first_epoch_rolled_back_keeps_factors():
    """A rate that overshoots: the first epoch is undone exactly (factors
    bitwise equal to the start), the rate is divided by ten and the index
    rewound; the next epochs proceed."""
    import torch
    print("case: rollback", flush=True)
    prob = gi.random_dense((9, 7, 40), 5, 3, "poisson_log", 3, dtype=np.float64)
    st, orc, T = _pair(prob, torch.float64, alpha_f=1.0, kappa_f=1)
    A0 = [a.clone() for a in st.factors()]
    st.update_factors(T(prob.X_t), T(prob.s_t))
    orc.update_factors(prob.X_t, prob.s_t)
    info = st.factor_info()
    assert orc.fac_info.rolled == [True] and info["rolled"] == [True]
    assert info["iters"] == 0 and info["alpha"] == pytest.approx(0.1)
    for a, b in zip(st.factors(), A0):
        assert torch.equal(a, b)


def test_tolerance_stops_before_any_iteration():
    import torch
    print("case: tol_f", flush=True)
    prob = gi.random_dense((9, 7, 40), 5, 3, "bernoulli_logit", 4, dtype=np.float64)
    st, orc, T = _pair(prob, torch.float64, alpha_f=0.1, tol_f=1e12)
    A0 = [a.clone() for a in st.factors()]
    st.update_factors(T(prob.X_t), T(prob.s_t))
    info = st.factor_info()
    assert info["epochs"] == 0 and info["iters"] == 0 and st.sync() == 0
    for a, b in zip(st.factors(), A0):
        assert torch.equal(a, b)


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log"])
def test_epochs_with_model_history(loss):
    """eq. gcp_stream_problem_2's history inside the epochs' objective."""
    import torch
    print("case: model history", loss, flush=True)
    prob = gi.random_dense((11, 6, 33), 4, 3, loss, 5, dtype=np.float64)
    st, orc, T = _pair(prob, torch.float64, hist="model", alpha_f=1.0)
    for step in range(2):
        st.update_factors(T(prob.X_t), T(prob.s_t))
        orc.update_factors(prob.X_t, prob.s_t)
        info = st.factor_info()
        assert _clear(orc.fac_info, 1e-10)
        assert info["rolled"] == orc.fac_info.rolled
        for k, a in enumerate(st.factors()):
            assert rel_err(a.cpu().numpy(), orc.A[k]) <= 1e-9


def test_online_gcp_steps_with_both_sgd_solvers():
    """Algorithm 1 with Algorithm 3 for s_t and Algorithm 4 for the factors:
    three time steps of a Poisson stream with new slices."""
    import torch
    print("case: online steps", flush=True)
    prob = gi.random_dense((10, 8, 50), 4, 2, "poisson_log", 6, dtype=np.float64)
    sgd = dict(tsolve="sgd", tau_w=5, kappa_w=3, alpha_w=0.05, alpha_f=0.2)
    st, orc, T = _pair(prob, torch.float64, **sgd)
    g = np.random.default_rng(9)
    for step in range(3):
        X = g.poisson(1.0, size=prob.dims).astype(np.float64)
        s = st.step(T(X))
        s_ref = orc.step(X)
        assert st.sync() == 0
        assert st.solve_info()["rolled"] == orc.solve_info.rolled
        assert st.factor_info()["rolled"] == orc.fac_info.rolled
        assert rel_err(s.cpu().numpy(), s_ref) <= 1e-9
        for k, a in enumerate(st.factors()):
            assert rel_err(a.cpu().numpy(), orc.A[k]) <= 1e-9, (step, k)
