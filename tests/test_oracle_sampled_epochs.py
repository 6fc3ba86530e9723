"""Pins of the oracle's Algorithm 4 on sparse slices with Algorithm 5's
objective estimates."""
from types import SimpleNamespace

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import sampled as osm
from oracle.adam import adam_step


def _state(prob, alpha):
    A = [np.asarray(a, np.float64).copy() for a in prob.A]
    z = [np.zeros_like(a) for a in A]
    return SimpleNamespace(A=A, u=[a.copy() for a in z], v=[a.copy() for a in z], Ao=[a.copy() for a in A],
                           uo=[a.copy() for a in z], vo=[a.copy() for a in z], alpha=alpha, i=0, call=0)


def _prob(seed=5):
    return gi.sparse_problem(dims=(12, 10, 9), rank=3, window=1, nnz=150, p=200, q=200, seed=seed,
                             loss="poisson_log")


def test_estimate_uses_fixed_draws_and_drops_mu():
    p = _prob()
    c = osm.estimate_call(p.t)
    a = osm.estimate_objective(p, 300, 300, c)
    assert osm.estimate_objective(p, 300, 300, c) == a
    p.mu = 5.0
    assert osm.estimate_objective(p, 300, 300, c) == a
    assert osm.estimate_objective(p, 300, 300, c + 1) != a
    assert c != 0 and osm.estimate_call(p.t + 1) != c


def test_estimate_is_unbiased():
    """E[F~] = F: the mean over many independent draw sets is within a
    CLT band of the exact objective of the dense equivalent (mu = 0)."""
    p = _prob(seed=7)
    vals = np.array([osm.estimate_objective(p, 100, 100, 1000 + k) for k in range(400)])
    # exact objective: data terms of each slice (zeros included) + lam term
    A = [np.asarray(a, np.float64) for a in p.A]
    F = 0.5 * p.lam * sum(np.sum(a * a) for a in A)
    for h, (sl, s) in enumerate([(p.X_t, p.s_t)] + list(zip(p.X_hist, p.s_hist))):
        X = np.zeros(p.dims)
        X[tuple(sl.coords.T)] = sl.vals
        c = 1.0 if h == 0 else p.w * p.theta ** (p.t - int(p.t_hist[h - 1]))
        F += c * np.sum(og.loss_f(p.loss, X, og.full_model(A, np.asarray(s, np.float64))))
    assert abs(vals.mean() - F) <= 4 * vals.std(ddof=1) / np.sqrt(len(vals))


def test_one_accepted_epoch_is_the_plain_iterations():
    p = _prob()
    st = _state(p, 1e-3)
    rolled = osm.sampled_factor_epochs(p, st, tau=2, kappa=1, p_est=300, q_est=300)
    assert rolled == [False]
    A = [np.asarray(a, np.float64).copy() for a in _prob().A]
    u = [np.zeros_like(a) for a in A]
    v = [np.zeros_like(a) for a in A]
    q = _prob()
    for it in range(2):
        q.A = A
        _, G, _ = osm.sampled_loss_grad(q, call=it)
        for k in range(3):
            A[k], u[k], v[k] = adam_step(A[k], G[k], u[k], v[k], it, 1e-3)
    for x, y in zip(st.A, A):
        assert np.array_equal(x, y)
    assert st.call == 2 and st.i == 2


def test_rolled_back_epoch_restores_and_keeps_counting_draws():
    p = _prob()
    st = _state(p, 3.0)
    A0 = [a.copy() for a in st.A]
    rolled = osm.sampled_factor_epochs(p, st, tau=2, kappa=1, p_est=300, q_est=300)
    assert rolled == [True]
    for x, y in zip(st.A, A0):
        assert np.array_equal(x, y)
    assert st.i == 0 and st.alpha == pytest.approx(0.3) and st.call == 2


def test_sampled_weight_solve_is_adam_on_the_sampled_weight_gradient():
    """Two accepted ADAM steps of Algorithm 3 on the sparse slice equal two
    ADAM steps on the (separately pinned) sampled weight gradient of X_t
    alone, calls 7 and 8, with the factor regulariser and history left out;
    the epoch is judged on the estimate with the weight solver's draws."""
    from types import SimpleNamespace
    p = _prob(seed=8)
    s, info = osm.sampled_temporal_sgd(p, 7, alpha=0.02, tau=2, kappa=1, p_est=300, q_est=300)
    q = SimpleNamespace(**vars(p))
    q.X_hist, q.s_hist, q.t_hist, q.lam = [], np.zeros((0, 3)), np.zeros(0, np.int64), 0.0
    ref, u, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for it, call in enumerate((7, 8)):
        q.s_t = ref
        g = osm.sampled_loss_grad(q, call=call)[2]
        ref, u, v = adam_step(ref, g, u, v, it, 0.02)
    F1 = osm.estimate_objective(SimpleNamespace(**{**vars(q), "s_t": ref, "mu": p.mu}), 300, 300,
                                osm.weight_estimate_call(p.t))
    assert info.F_try[0] == pytest.approx(F1 + 0.5 * p.mu * float(ref @ ref), rel=1e-14)
    if info.rolled == [False]:
        assert np.array_equal(s, ref)
    assert info.call == 9


def test_sampled_weight_solve_draws_differ_from_the_factor_estimates():
    p = _prob()
    assert osm.weight_estimate_call(p.t) != osm.estimate_call(p.t)
    assert osm.weight_estimate_call(p.t) != osm.weight_estimate_call(p.t + 1)
