"""FP64 oracle for the ADAM step of Algorithm 2 (Step method).

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

    u <- b1 u + (1-b1) g ;  v <- b2 v + (1-b2) g^2
    alpha~ = alpha sqrt(1 - b2^n) / (1 - b1^n)
    a <- max(a - alpha~ u / (sqrt(v) + eps), l)

Reading: Algorithm 1 starts the iteration index at 0 while the bias
correction divides by 1 - b1^i, which is zero at i = 0; the standard 1-based
step n = i + 1 is used.
"""
import math

import numpy as np


def adam_step(a, g, u, v, i: int, alpha: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, lower: float = -np.inf):
    """Returns (a_new, u_new, v_new) for global iteration index i."""
    a = np.asarray(a, np.float64)
    g = np.asarray(g, np.float64)
    u = beta1 * np.asarray(u, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    n = i + 1
    alpha_t = alpha * math.sqrt(1.0 - beta2 ** n) / (1.0 - beta1 ** n)
    a_new = np.maximum(a - alpha_t * u / (np.sqrt(v) + eps), lower)
    return a_new, u, v
