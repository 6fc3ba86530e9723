"""Pins of the oracle's Algorithm 4 epochs (with the ADAM Update of
Algorithm 2) against the plain iterations they are built from."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle.stream import StreamOracle
from oracle.temporal_sgd import DECAY


def _oracle(prob, **kw):
    base = dict(loss=prob.loss, window=len(prob.X_hist), w=1.1, theta=0.9, lam=0.05, mu=0.3, tau_f=3, seed=2)
    base.update(kw)
    return StreamOracle(prob.A, prob.X_hist, prob.s_hist, prob.t_hist, **base)


def _prob(loss="poisson_log", seed=1):
    return gi.random_dense((4, 5, 6), 3, 2, loss, seed, dtype=np.float64)


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
def test_one_accepted_epoch_is_the_plain_iterations(loss):
    p = _prob(loss)
    a = _oracle(p, alpha_f=1e-3)
    b = _oracle(p, alpha_f=1e-3, kappa_f=1)
    a.update_factors(p.X_t, p.s_t)
    b.update_factors(p.X_t, p.s_t)
    assert b.fac_info.rolled == [False]
    for x, y in zip(a.A, b.A):
        assert np.array_equal(x, y)
    assert a.i == b.i == 3


def test_rolled_back_epoch_restores_and_decays():
    p = _prob()
    o = _oracle(p, alpha_f=2.0, kappa_f=1)
    A0 = [a.copy() for a in o.A]
    o.update_factors(p.X_t, p.s_t)
    assert o.fac_info.rolled == [True]
    assert o.fac_info.F_try[0] > o.fac_info.F[0] == o.fac_info.F[1]
    for x, y in zip(o.A, A0):
        assert np.array_equal(x, y)
    assert all(not np.any(u) for u in o.u) and o.i == 0
    assert o.alpha_f == 2.0 * DECAY


def test_rate_persists_across_time_steps():
    """The factor ADAM object lives for the whole stream (Algorithm 1 creates
    it once): a decayed rate is not reset by the next time step."""
    p = _prob()
    o = _oracle(p, alpha_f=2.0, kappa_f=1)
    o.update_factors(p.X_t, p.s_t)
    assert o.alpha_f == 2.0 * DECAY
    o.update_factors(p.X_t, p.s_t)
    assert o.alpha_f in (2.0 * DECAY, 2.0 * DECAY * DECAY)


def test_accepted_epochs_never_increase_the_objective():
    p = _prob("bernoulli_logit", seed=4)
    o = _oracle(p, alpha_f=0.3, kappa_f=8)
    o.update_factors(p.X_t, p.s_t)
    F = o.fac_info.F
    assert all(b <= a for a, b in zip(F, F[1:]))
    assert o.i == 3 * sum(not r for r in o.fac_info.rolled)


def test_tolerance_stops_before_any_iteration():
    p = _prob()
    o = _oracle(p, alpha_f=1e-2, kappa_f=5, tol_f=1e12)
    A0 = [a.copy() for a in o.A]
    o.update_factors(p.X_t, p.s_t)
    assert o.fac_info.rolled == [] and o.i == 0
    for x, y in zip(o.A, A0):
        assert np.array_equal(x, y)


def test_factor_objective_leaves_out_the_weight_regulariser():
    """Algorithm 4 estimates the objective with mu = 0."""
    p = _prob()
    a = _oracle(p, mu=0.0)
    b = _oracle(p, mu=7.0)
    assert a.factor_objective(p.X_t, p.s_t) == b.factor_objective(p.X_t, p.s_t)
