"""FP64 oracle for the model-difference history of eq. gcp_stream_problem_2.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).  Shares no
code with the HIP library.

In this formulation (Section 4.1) the window keeps only the temporal weights
s_h of past slices, not the slices.  The history term compares the CP model
built from the previous step's factors Abar with the one built from the
current factors A, both with the stored weight s_h:

  F = sum_i f(x_it, m_i(s_t)) + 1/2 sum_h w_h ||Mbar_h - M_h||_F^2
      + lam/2 sum_k ||A^(k)||_F^2 + mu/2 ||s_t||^2,
  Mbar_h = [[Abar; s_h]],  M_h = [[A; s_h]],  w_h = w theta^(t-h),

and its factor gradient is eq. spatial_gcp_grad (Section 4.2):

  dF/dA^(k) = Y_t(k) Z_k diag(s_t) + lam A^(k)
      + sum_h w_h (A^(k) diag(s_h) Z_k^T Z_k diag(s_h)
                   - Abar^(k) diag(s_h) Zbar_k^T Z_k diag(s_h)).

The weight gradient is that of the single-slice problem: the history term
does not depend on s_t.  Everything below is the definition written out:
dense models, explicit Khatri-Rao products.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .gcp import full_model, gradient, history_weights, objective, z_except


def history_objective(A: Sequence[np.ndarray], A_old: Sequence[np.ndarray], s_hist, c_hist) -> float:
    """1/2 sum_h w_h ||Mbar_h - M_h||_F^2 with dense models."""
    A = [np.asarray(a, np.float64) for a in A]
    Ab = [np.asarray(a, np.float64) for a in A_old]
    F = 0.0
    for s, c in zip(np.asarray(s_hist, np.float64).reshape(len(c_hist), -1), c_hist):
        D = full_model(Ab, s) - full_model(A, s)
        F += 0.5 * float(c) * float(np.sum(D * D))
    return F


def history_gradient(A: Sequence[np.ndarray], A_old: Sequence[np.ndarray], s_hist, c_hist):
    """The history part of eq. spatial_gcp_grad, with Z_k and Zbar_k as
    explicit Khatri-Rao products."""
    A = [np.asarray(a, np.float64) for a in A]
    Ab = [np.asarray(a, np.float64) for a in A_old]
    G = [np.zeros_like(a) for a in A]
    for s, c in zip(np.asarray(s_hist, np.float64).reshape(len(c_hist), -1), c_hist):
        Ds = np.diag(s)
        for k in range(len(A)):
            Zk = z_except(A, k)
            Zbk = z_except(Ab, k)
            G[k] += float(c) * (A[k] @ Ds @ (Zk.T @ Zk) @ Ds - Ab[k] @ Ds @ (Zbk.T @ Zk) @ Ds)
    return G


def _current_only(prob):
    """The problem with its window emptied: the data term of X_t alone."""
    from types import SimpleNamespace
    return SimpleNamespace(X_t=prob.X_t, A=prob.A, s_t=prob.s_t, X_hist=[],
                           s_hist=np.zeros((0, len(prob.s_t))), t_hist=np.zeros(0, np.int64),
                           t=prob.t, w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu,
                           loss=prob.loss)


def objective_model(prob) -> float:
    """F of eq. gcp_stream_problem_2.  prob carries A_old, s_hist, t_hist."""
    c = history_weights(prob.t, prob.t_hist, prob.w, prob.theta)
    return objective(_current_only(prob)) + history_objective(prob.A, prob.A_old, prob.s_hist, c)


def gradient_model(prob):
    """(G^(1..d), g_s) of eq. gcp_stream_problem_2."""
    c = history_weights(prob.t, prob.t_hist, prob.w, prob.theta)
    G, g_s = gradient(_current_only(prob))
    Gh = history_gradient(prob.A, prob.A_old, prob.s_hist, c)
    return [g + h for g, h in zip(G, Gh)], g_s
