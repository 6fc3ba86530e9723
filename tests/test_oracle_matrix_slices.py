"""Pins of the matrix-slice (d = 2) reading: the d = 3 problem with I3 = 1
and a fixed row of ones has the two-way model, objective and gradients."""
import numpy as np
import pytest

from oracle import gcp as og
from oracle.stream import StreamOracle


@pytest.mark.parametrize("loss", og.LOSSES)
def test_two_way_objective_and_gradient(loss):
    g = np.random.default_rng(3)
    I, J, R, lam, mu = 7, 5, 3, 0.3, 0.2
    A, B = g.uniform(-0.6, 0.6, (I, R)), g.uniform(-0.6, 0.6, (J, R))
    s = g.uniform(0.5, 1.5, R)
    X = g.poisson(1.0, (I, J)).astype(float) if loss != "gaussian" else g.normal(size=(I, J))
    if loss == "bernoulli_logit":
        X = (X > 0).astype(float)
    orc = StreamOracle([A, B], [], np.zeros((0, R)), [], loss=loss, lam=lam, mu=mu, d=2)
    # two-way formulas, written directly
    M = A @ np.diag(s) @ B.T
    Y = og.loss_dfdm(loss, X, M)
    F2 = np.sum(og.loss_f(loss, X, M)) + 0.5 * lam * (np.sum(A * A) + np.sum(B * B))
    GA = Y @ B @ np.diag(s) + lam * A
    GB = Y.T @ A @ np.diag(s) + lam * B
    gs = np.einsum("ir,ij,jr->r", A, Y, B) + mu * s
    assert orc.factor_objective(X, s) == pytest.approx(F2, rel=1e-13)
    prob = orc.problem(X.reshape(I, J, 1), s)
    G, g_s = og.gradient(prob)
    assert np.allclose(G[0], GA, rtol=1e-12, atol=1e-14) and np.allclose(G[1], GB, rtol=1e-12, atol=1e-14)
    assert np.allclose(g_s, gs, rtol=1e-12, atol=1e-14)


def test_fixed_row_never_moves():
    g = np.random.default_rng(4)
    A, B = g.uniform(-0.5, 0.5, (6, 2)), g.uniform(-0.5, 0.5, (4, 2))
    orc = StreamOracle([A, B], [], np.zeros((0, 2)), [], loss="gaussian", window=2, alpha_f=0.1, tau_f=3, d=2)
    for _ in range(3):
        orc.update_factors(g.normal(size=(6, 4)), np.ones(2))
    assert np.array_equal(orc.A[2], np.ones((1, 2))) and not np.array_equal(orc.A[0], A)
