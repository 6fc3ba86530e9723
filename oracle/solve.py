"""FP64 oracle for the least-squares temporal-weight solve.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

For the Gaussian loss the temporal subproblem (eq.
gcp_stream_temporal_problem, Section 4.2) is
    min_s  sum_i (x_it - m_i(s))^2 + mu/2 ||s||^2,   m = Z s,
and Section 5 replaces its SGD solver by one least-squares solve.  Setting the
derivative to zero gives (Z^T Z + mu/2 I) s = Z^T vec(X_t).  The solution is
computed here straight from that definition: Z is formed explicitly and the
normal equations are solved with numpy.linalg.solve.  Reading for the lower
bound l (the paper is silent about l with the LS solve): clamp after the
solve, s <- max(s, l).
"""
import numpy as np

from .gcp import vec, z_all


def ls_temporal(X_t, A, mu: float = 0.0, lower: float = -np.inf) -> np.ndarray:
    A = [np.asarray(a, np.float64) for a in A]
    Z = z_all(A)
    R = Z.shape[1]
    lhs = Z.T @ Z + 0.5 * mu * np.eye(R)
    rhs = Z.T @ vec(np.asarray(X_t, np.float64))
    s = np.linalg.solve(lhs, rhs)
    return np.maximum(s, lower)
