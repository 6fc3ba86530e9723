"""Pins of the temporal-weight GCP-SGD oracle (Algorithm 3 with the ADAM
Step/Update of Algorithm 2)."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import solve as osv
from oracle import temporal_sgd as ts


def test_gaussian_sgd_reaches_the_least_squares_weights():
    """The Gaussian temporal subproblem is a convex quadratic whose minimiser
    is the least-squares solve of Section 5; enough ADAM iterations reach it."""
    p = gi.random_dense((6, 7, 8), 3, 0, "gaussian", seed=1).promoted()
    s, info = ts.temporal_sgd(p.X_t, p.A, "gaussian", mu=0.2, alpha=0.02, tau=200, kappa=20)
    s_ls = osv.ls_temporal(p.X_t, p.A, mu=0.2)
    assert np.linalg.norm(s - s_ls) <= 1e-4 * np.linalg.norm(s_ls)
    assert all(b <= a for a, b in zip(info.F, info.F[1:]))


def test_rollback_restores_the_saved_state_and_decays_the_rate():
    """An epoch that raises the objective is undone: s and the moments return
    to the last accepted values, the rate is decreased, the count rewinds."""
    p = gi.random_dense((5, 6, 7), 3, 0, "poisson_log", seed=2).promoted()
    s, info = ts.temporal_sgd(p.X_t, p.A, "poisson_log", mu=0.1, alpha=50.0, tau=5, kappa=3)
    assert info.rolled[0]
    assert info.F[1] == info.F[0]
    assert info.alpha < 50.0
    if all(info.rolled):
        assert np.all(s == 0.0) and info.iters == 0


def test_objective_never_increases_and_bound_holds():
    p = gi.random_dense((6, 5, 4), 4, 0, "bernoulli_logit", seed=3).promoted()
    s, info = ts.temporal_sgd(p.X_t, p.A, "bernoulli_logit", mu=0.05, lower=0.0, alpha=0.5, tau=10, kappa=6)
    assert all(b <= a for a, b in zip(info.F, info.F[1:]))
    assert np.all(s >= 0.0)


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
def test_weight_gradient_matches_central_differences(loss):
    p = gi.random_dense((4, 5, 3), 3, 0, loss, seed=4).promoted()
    s = np.array([0.7, -0.2, 1.1])
    g = ts.weight_gradient(p.X_t, p.A, s, loss, 0.3)
    eps = 1e-6
    for j in range(3):
        sp, sm = s.copy(), s.copy()
        sp[j] += eps
        sm[j] -= eps
        fd = (ts.weight_objective(p.X_t, p.A, sp, loss, 0.3) - ts.weight_objective(p.X_t, p.A, sm, loss, 0.3)) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j]))
