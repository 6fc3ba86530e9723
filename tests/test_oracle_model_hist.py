"""Pins of the model-difference history oracle (eq. gcp_stream_problem_2):
a closed form through Gram matrices, central differences, the unfolding form
of the gradient, and the special cases that must vanish."""
import numpy as np
import pytest

from oracle import gcp as og
from oracle import model_hist as mh


def _setup(seed=0, dims=(4, 5, 3), R=3, H=2, drift=0.1):
    rng = np.random.default_rng(seed)
    A = [rng.normal(size=(n, R)) for n in dims]
    Ab = [a + drift * rng.normal(size=a.shape) for a in A]
    S = rng.uniform(0.5, 1.5, size=(H, R))
    c = rng.uniform(0.5, 1.5, size=H)
    return A, Ab, S, c


def test_objective_equals_gram_closed_form():
    """||Mbar - M||^2 = s'(*AbAb)s - 2 s'(*AbA)s + s'(*AA)s, with * the
    Hadamard product of the mode Gram matrices (derived, not printed)."""
    A, Ab, S, c = _setup(1)
    want = 0.0
    for s, w in zip(S, c):
        P = np.prod([a.T @ a for a in A], axis=0)
        Q = np.prod([b.T @ a for a, b in zip(A, Ab)], axis=0)
        O = np.prod([b.T @ b for b in Ab], axis=0)
        want += 0.5 * w * (s @ O @ s - 2 * s @ Q @ s + s @ P @ s)
    got = mh.history_objective(A, Ab, S, c)
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_gradient_matches_central_differences():
    A, Ab, S, c = _setup(2)
    G = mh.history_gradient(A, Ab, S, c)
    eps = 1e-6
    for k in range(3):
        fd = np.zeros_like(A[k])
        for idx in np.ndindex(*A[k].shape):
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[k][idx] += eps
            Am[k][idx] -= eps
            fd[idx] = (mh.history_objective(Ap, Ab, S, c) - mh.history_objective(Am, Ab, S, c)) / (2 * eps)
        assert np.max(np.abs(fd - G[k])) <= 1e-7 * max(1.0, np.max(np.abs(G[k])))


def test_gradient_equals_unfolding_form():
    """d/dA^(k) of 1/2 ||Mbar - M||^2 = -(Mbar - M)_(k) Z_k diag(s)."""
    A, Ab, S, c = _setup(3, dims=(3, 4, 5), R=4, H=3)
    G = mh.history_gradient(A, Ab, S, c)
    for k in range(3):
        want = np.zeros_like(A[k])
        for s, w in zip(S, c):
            D = og.full_model(Ab, s) - og.full_model(A, s)
            want -= w * (og.unfold(D, k) @ og.z_except(A, k)) * s[None, :]
        assert np.allclose(G[k], want, rtol=1e-12, atol=1e-12)


def test_unchanged_factors_give_no_history_term():
    A, _, S, c = _setup(4)
    assert mh.history_objective(A, A, S, c) == 0.0
    for g in mh.history_gradient(A, A, S, c):
        assert np.all(g == 0.0)


@pytest.mark.parametrize("loss", og.LOSSES)
def test_full_gradient_matches_central_differences(loss):
    """Data term of X_t plus the history term, every factor entry and s_t."""
    from types import SimpleNamespace
    A, Ab, S, _ = _setup(5, dims=(3, 4, 2), R=2, H=2)
    rng = np.random.default_rng(6)
    X = (rng.poisson(1.0, size=(3, 4, 2)) if loss == "poisson_log" else
         (rng.random((3, 4, 2)) < 0.4) if loss == "bernoulli_logit" else
         rng.normal(size=(3, 4, 2))).astype(np.float64)
    prob = SimpleNamespace(X_t=X, A=A, A_old=Ab, s_t=rng.uniform(0.5, 1.5, 2), s_hist=S,
                           t_hist=np.array([2, 4]), t=6, w=1.2, theta=0.8, lam=0.1, mu=0.2, loss=loss)
    G, g_s = mh.gradient_model(prob)
    eps = 1e-6

    def F_with(Ak=None, k=None, s=None):
        q = SimpleNamespace(**vars(prob))
        if Ak is not None:
            q.A = [a if l != k else Ak for l, a in enumerate(A)]
        if s is not None:
            q.s_t = s
        return mh.objective_model(q)

    for k in range(3):
        for idx in np.ndindex(*A[k].shape):
            Ap, Am = A[k].copy(), A[k].copy()
            Ap[idx] += eps
            Am[idx] -= eps
            fd = (F_with(Ap, k) - F_with(Am, k)) / (2 * eps)
            assert abs(fd - G[k][idx]) <= 1e-6 * max(1.0, abs(G[k][idx]))
    for j in range(2):
        sp, sm = prob.s_t.copy(), prob.s_t.copy()
        sp[j] += eps
        sm[j] -= eps
        fd = (F_with(s=sp) - F_with(s=sm)) / (2 * eps)
        assert abs(fd - g_s[j]) <= 1e-6 * max(1.0, abs(g_s[j]))
