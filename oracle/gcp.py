"""FP64 CPU oracle for the streaming GCP objective and gradient.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
module: only the tests, the smoke check and the bench's CPU-baseline leg use
it.  It shares no code with the HIP library.

Two tiers compute the same quantities:

* tier V (vectorised NumPy) writes the paper's formulas literally: the CP
  model of eq. CP_model, the gradient tensor Y of Section 2.2, and the factor
  and weight gradients of eqs. gcp_grad_A / gcp_grad_lambda using the mode-k
  unfolding Y_(k) and the Khatri-Rao products Z_k and Z;
* tier L (pure Python loops over every multi-index) writes the same sums
  index by index and serves tiny inputs only.

The objective is the single-slice problem with the stored-slice history term
of eq. gcp_stream_problem_1 (Section 4.1):

  F = sum_i f(x_it, m_i(s_t)) + sum_h w_h sum_i f(x_ih, m_i(s_h))
      + lam/2 sum_k ||A^(k)||_F^2 + mu/2 ||s_t||^2,   w_h = w theta^(t-h)

where the historical model uses the stored weight s_h with the *current*
factor matrices.  Readings taken where the paper is silent or inconsistent:

* Losses (Section 2.2 defines f = -log p(x | l^-1(m))): Gaussian
  f = (x-m)^2 exactly as printed (no 1/2); Poisson with log link
  f = exp(m) - x m; Bernoulli with logit link f = log(1+exp(m)) - x m.  Terms
  that do not depend on m are dropped.
* The temporal-weight gradient of Section 4.2 prints lambda for the
  regulariser; the temporal subproblem (eq. gcp_stream_temporal_problem)
  uses mu, which is what its derivative gives, so mu is used.
* Only the current slice contributes to the weight gradient: s_h is fixed.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Sequence

import numpy as np

LOSSES = ("gaussian", "poisson_log", "bernoulli_logit")
# The two losses Section 2.2 writes out (identity and odds links), defined
# for m >= 0, with log m replaced by log(m + eps) as its footnote says; the
# paper leaves eps open ("a small constant"): 1e-10 here.
PAPER_LOSSES = ("poisson_id", "bernoulli_odds")
EPS = 1e-10


# ------------------------------------------------------------- losses ----
def loss_f(loss: str, x, m):
    """Elementwise loss f(x, m) (Section 2.2, log/logit links)."""
    x = np.asarray(x, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    if loss == "gaussian":
        return (x - m) ** 2
    if loss == "poisson_log":
        return np.exp(m) - x * m
    if loss == "bernoulli_logit":
        # log(1 + e^m) written so that it neither overflows nor cancels
        return np.maximum(m, 0.0) + np.log1p(np.exp(-np.abs(m))) - x * m
    if loss == "poisson_id":
        return m - x * np.log(m + EPS)
    if loss == "bernoulli_odds":
        return np.log1p(m) - x * np.log(m + EPS)
    raise ValueError(loss)


def loss_dfdm(loss: str, x, m):
    """Elementwise derivative y = df/dm (Section 2.2)."""
    x = np.asarray(x, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    if loss == "gaussian":
        return 2.0 * (m - x)
    if loss == "poisson_log":
        return np.exp(m) - x
    if loss == "bernoulli_logit":
        e = np.exp(-np.abs(m))
        sig = np.where(m >= 0, 1.0 / (1.0 + e), e / (1.0 + e))
        return sig - x
    if loss == "poisson_id":
        return 1.0 - x / (m + EPS)
    if loss == "bernoulli_odds":
        return 1.0 / (m + 1.0) - x / (m + EPS)
    raise ValueError(loss)


# -------------------------------------------------- tensor algebra ------
def unfold(X: np.ndarray, k: int) -> np.ndarray:
    """Mode-k matricization X_(k) (Kolda-Bader convention): rows are i_k,
    columns enumerate the other indices with the lowest mode fastest."""
    d = X.ndim
    others = [l for l in range(d) if l != k]
    return X.transpose([k] + others[::-1]).reshape(X.shape[k], -1)


def vec(X: np.ndarray) -> np.ndarray:
    """Column-major vectorisation (i_1 fastest), matching Z's row order."""
    return X.transpose(list(range(X.ndim))[::-1]).reshape(-1)


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """B_1 (.) B_2 (.) ... : column-wise Kronecker, the last factor's row
    index runs fastest."""
    out = mats[0]
    for b in mats[1:]:
        R = out.shape[1]
        out = (out[:, None, :] * b[None, :, :]).reshape(-1, R)
    return out


def z_all(A: Sequence[np.ndarray]) -> np.ndarray:
    """Z = A^(d) (.) ... (.) A^(1)."""
    return khatri_rao(list(A)[::-1])


def z_except(A: Sequence[np.ndarray], k: int) -> np.ndarray:
    """Z_k = A^(d) (.) .. A^(k+1) (.) A^(k-1) (.) .. A^(1)."""
    return khatri_rao([A[l] for l in range(len(A) - 1, -1, -1) if l != k])


def full_model(A: Sequence[np.ndarray], s: np.ndarray) -> np.ndarray:
    """M = sum_j s_j a_j^(1) o ... o a_j^(d)  (eq. CP_model)."""
    dims = tuple(a.shape[0] for a in A)
    M = np.zeros(dims)
    for j in range(len(s)):
        comp = s[j] * A[0][:, j]
        for a in A[1:]:
            comp = np.multiply.outer(comp, a[:, j])
        M += comp
    return M


def history_weights(t: int, t_hist, w: float, theta: float) -> np.ndarray:
    """w_h = w theta^(t-h)  (Section 4.1)."""
    return np.array([w * theta ** (t - int(h)) for h in t_hist], dtype=np.float64)


def _slices(prob):
    """(X, s, c) for the current slice (c = 1) then each stored slice."""
    c_hist = history_weights(prob.t, prob.t_hist, prob.w, prob.theta)
    out = [(np.asarray(prob.X_t, np.float64), np.asarray(prob.s_t, np.float64), 1.0)]
    for h in range(len(prob.X_hist)):
        out.append((np.asarray(prob.X_hist[h], np.float64),
                    np.asarray(prob.s_hist[h], np.float64), float(c_hist[h])))
    return out


def _regulariser(prob, A) -> float:
    return (0.5 * prob.lam * sum(float(np.sum(a * a)) for a in A)
            + 0.5 * prob.mu * float(np.sum(np.asarray(prob.s_t, np.float64) ** 2)))


# ------------------------------------------------------------ tier V ----
def objective(prob) -> float:
    """F of eq. gcp_stream_problem_1 (stored-slice history)."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    F = 0.0
    for X, s, c in _slices(prob):
        F += c * float(np.sum(loss_f(prob.loss, X, full_model(A, s))))
    return F + _regulariser(prob, A)


def gradient(prob):
    """(G^(1..d), g_s): eq. gcp_grad_A per slice with diag(s_h) and weight
    w_h, plus lam A^(k); eq. gcp_grad_lambda on the current slice plus mu s_t
    (Section 4.2)."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    d = len(A)
    G = [prob.lam * a.copy() for a in A]
    g_s = None
    for n, (X, s, c) in enumerate(_slices(prob)):
        Y = loss_dfdm(prob.loss, X, full_model(A, s))
        for k in range(d):
            G[k] += c * (unfold(Y, k) @ z_except(A, k)) * s[None, :]
        if n == 0:
            g_s = z_all(A).T @ vec(Y) + prob.mu * np.asarray(prob.s_t, np.float64)
    return G, g_s


def loss_terms_abs(prob) -> float:
    """sum of |c_h f| over every entry-slice: the scale against which the
    objective's rounding error is measured (it can cross zero)."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    tot = 0.0
    for X, s, c in _slices(prob):
        tot += abs(c) * float(np.sum(np.abs(loss_f(prob.loss, X, full_model(A, s)))))
    return tot + abs(_regulariser(prob, A))


# ------------------------------------------------------------ tier L ----
def _m_loop(A, s, idx) -> float:
    m = 0.0
    for j in range(len(s)):
        p = float(s[j])
        for k, ik in enumerate(idx):
            p *= float(A[k][ik, j])
        m += p
    return m


def objective_loops(prob) -> float:
    """Tier L: the objective by explicit summation over every multi-index."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    dims = tuple(a.shape[0] for a in A)
    F = 0.0
    for X, s, c in _slices(prob):
        for idx in itertools.product(*[range(n) for n in dims]):
            F += c * float(loss_f(prob.loss, X[idx], _m_loop(A, s, idx)))
    for a in A:
        for v in a.ravel():
            F += 0.5 * prob.lam * float(v) * float(v)
    for v in np.asarray(prob.s_t, np.float64):
        F += 0.5 * prob.mu * float(v) * float(v)
    return F


def gradient_loops(prob):
    """Tier L: G^(k)[r,j] = sum_{i: i_k=r} sum_h c_h y_ih s_hj prod_{l!=k}
    A^(l)[i_l,j] + lam A^(k)[r,j];  g_s[j] = sum_i y_it prod_k A^(k)[i_k,j]
    + mu s_tj."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    d = len(A)
    dims = tuple(a.shape[0] for a in A)
    R = A[0].shape[1]
    G = [np.zeros_like(a) for a in A]
    g_s = np.zeros(R)
    for n, (X, s, c) in enumerate(_slices(prob)):
        for idx in itertools.product(*[range(nn) for nn in dims]):
            y = float(loss_dfdm(prob.loss, X[idx], _m_loop(A, s, idx)))
            for j in range(R):
                for k in range(d):
                    p = 1.0
                    for l in range(d):
                        if l != k:
                            p *= float(A[l][idx[l], j])
                    G[k][idx[k], j] += c * y * float(s[j]) * p
                if n == 0:
                    p = 1.0
                    for l in range(d):
                        p *= float(A[l][idx[l], j])
                    g_s[j] += y * p
    for k in range(d):
        G[k] += prob.lam * A[k]
    g_s += prob.mu * np.asarray(prob.s_t, np.float64)
    return G, g_s
