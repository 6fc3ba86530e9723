"""FP64 oracle for the temporal-weight GCP-SGD solver (Algorithm 3) with the
ADAM Step and Update methods of Algorithm 2.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

For dense slices the objective estimate and the stochastic gradient of the
algorithm are taken exactly: the objective of X_t alone,
    F(s) = sum_i f(x_it, m_i(s)) + mu/2 ||s||^2
(the history and factor terms do not depend on s, eq.
gcp_stream_temporal_problem), and its gradient Z' vec(Y) + mu s.  The steps,
in the algorithm's order:

  s <- 0; reset the ADAM moments and the saved copies; F <- F(s); i <- 0
  while F > tol_w, for at most kappa_w epochs:
      F_old <- F
      tau_w times: s <- Step(s, grad F(s), i); i <- i + 1
      F <- F(s)
      if F > F_old: roll back s and the moments to the saved copies,
                    decrease the rate, F <- F_old, i <- i - tau_w
      else:         save s and the moments

Readings (the paper leaves these open): the regulariser of the weight
gradient is mu (the printed lambda is the factor one; the subproblem's own
derivative gives mu); "decrease the learning rate" multiplies it by
decay = 0.1; the Step's bias correction uses the 1-based step i + 1.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from .adam import adam_step
from .gcp import gradient, objective

DECAY = 0.1


def _problem(X_t, A, s, loss, mu):
    R = A[0].shape[1]
    return SimpleNamespace(X_t=np.asarray(X_t, np.float64), A=[np.asarray(a, np.float64) for a in A],
                           s_t=np.asarray(s, np.float64), X_hist=[], s_hist=np.zeros((0, R)),
                           t_hist=np.zeros(0, np.int64), t=1, w=1.0, theta=1.0, lam=0.0, mu=mu, loss=loss)


def weight_objective(X_t, A, s, loss, mu) -> float:
    return objective(_problem(X_t, A, s, loss, mu))


def weight_gradient(X_t, A, s, loss, mu) -> np.ndarray:
    return gradient(_problem(X_t, A, s, loss, mu))[1]


def temporal_sgd(X_t, A, loss, *, mu=0.0, lower=-np.inf, alpha=1e-3, tau=10, kappa=5, tol=-np.inf,
                 beta1=0.9, beta2=0.999, eps=1e-8):
    """Algorithm 3 with exact objective and gradient.  Returns (s, info):
    info.F holds the accepted objective before the first epoch and after
    each one, info.F_try the objective each epoch reached before its
    decision, info.rolled the decisions."""
    R = np.asarray(A[0]).shape[1]
    s = np.zeros(R)
    u = np.zeros(R)
    v = np.zeros(R)
    s_o, u_o, v_o = s.copy(), u.copy(), v.copy()
    F = weight_objective(X_t, A, s, loss, mu)
    i = 0
    hist, tried, rolled = [F], [], []
    for _ in range(kappa):
        if not F > tol:
            break
        F_old = F
        for _ in range(tau):
            g = weight_gradient(X_t, A, s, loss, mu)
            s, u, v = adam_step(s, g, u, v, i, alpha, beta1, beta2, eps, lower)
            i += 1
        F = weight_objective(X_t, A, s, loss, mu)
        tried.append(F)
        if F > F_old:
            s, u, v = s_o.copy(), u_o.copy(), v_o.copy()
            alpha *= DECAY
            F = F_old
            i -= tau
            rolled.append(True)
        else:
            s_o, u_o, v_o = s.copy(), u.copy(), v.copy()
            rolled.append(False)
        hist.append(F)
    return s, SimpleNamespace(F=hist, F_try=tried, rolled=rolled, alpha=alpha, iters=i)
