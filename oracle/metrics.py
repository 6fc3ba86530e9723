"""FP64 oracle for the evaluation metrics of Section 6.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

* Local reconstruction loss (eq. local_loss): the loss of a slice under the
  CP model with the current factors and that slice's weights, over the
  squared Frobenius norm of the slice:  F_local = sum_i f(x_i, m_i) / ||X||_F^2.
  The global loss has the same form with the final factors, summed over all
  past slices: sum_t sum_i f(x_it, m_it) / sum_t ||X_t||_F^2 (reading: one
  ratio of sums, as for a tensor of stacked slices).
* K-tensor score (the congruence of Section 6.1 between a computed and a
  planted K-tensor, 1.0 for perfect recovery).  Reading, following the
  congruence measure the paper cites: normalise every factor column, move the
  norms into the component weights, and score a pair of components (r, q) as
      (1 - |xi_r - eta_q| / max(xi_r, eta_q)) * prod_k |a_r^(k)' b_q^(k)|;
  components are matched greedily (highest pair score first, each component
  used once) and the score is the mean over the R matched pairs of the
  reference.
"""
from __future__ import annotations

import numpy as np

from .gcp import full_model, loss_f


def slice_loss(X, A, s, loss):
    """(sum_i f(x_i, m_i), ||X||_F^2) for one slice."""
    X = np.asarray(X, np.float64)
    M = full_model([np.asarray(a, np.float64) for a in A], np.asarray(s, np.float64))
    return float(np.sum(loss_f(loss, X, M))), float(np.sum(X * X))


def local_loss(X, A, s, loss) -> float:
    f, n2 = slice_loss(X, A, s, loss)
    return f / n2


def global_loss(Xs, A, S, loss) -> float:
    parts = [slice_loss(X, A, s, loss) for X, s in zip(Xs, S)]
    return sum(p[0] for p in parts) / sum(p[1] for p in parts)


def _normalise(A, w):
    A = [np.asarray(a, np.float64) for a in A]
    w = np.asarray(w, np.float64).copy()
    U = []
    for a in A:
        n = np.linalg.norm(a, axis=0)
        w = w * n
        U.append(a / np.where(n > 0, n, 1.0))
    return U, w


def pair_scores(A, wa, B, wb) -> np.ndarray:
    """R_a x R_b matrix of component-pair scores."""
    Ua, xi = _normalise(A, wa)
    Ub, eta = _normalise(B, wb)
    C = np.ones((Ua[0].shape[1], Ub[0].shape[1]))
    for a, b in zip(Ua, Ub):
        C *= np.abs(a.T @ b)
    big = np.maximum(np.abs(xi)[:, None], np.abs(eta)[None, :])
    pen = 1.0 - np.abs(np.abs(xi)[:, None] - np.abs(eta)[None, :]) / np.where(big > 0, big, 1.0)
    return C * pen


def ktensor_score(A, wa, B, wb) -> float:
    """Greedy-matched mean pair score of K-tensor (A, wa) against the
    reference (B, wb)."""
    P = pair_scores(A, wa, B, wb)
    Ra, Rb = P.shape
    used_a, used_b, total = set(), set(), 0.0
    order = sorted(((P[i, j], i, j) for i in range(Ra) for j in range(Rb)), key=lambda t: (-t[0], t[1], t[2]))
    for v, i, j in order:
        if i in used_a or j in used_b:
            continue
        used_a.add(i)
        used_b.add(j)
        total += v
        if len(used_b) == min(Ra, Rb):
            break
    return total / Rb
