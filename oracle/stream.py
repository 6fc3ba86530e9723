"""FP64 oracle for one OnlineGCP time step on dense slices.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

Follows the body of Algorithm 1 (Section 4.3) in the paper's order:
  1. A <- A_old;
  2. the temporal weights s_t: the Gaussian least-squares solve that Section
     5 allows in place of Algorithm 3 (see solve.py), or with tsolve="sgd"
     Algorithm 3 itself (see temporal_sgd.py);
  3. the factor update: tau_f iterations of Algorithm 4's inner loop, each a
     full gradient of eq. gcp_stream_problem_1 (stored-slice history, see
     gcp.py) followed by the ADAM Step of Algorithm 2 with the global
     iteration index i carried across slices; with kappa_f > 0, Algorithm 4's
     epochs: at most kappa_f epochs of tau_f iterations while F > tol_f, each
     followed by the objective, and the ADAM Update of Algorithm 2 (keep the
     epoch, or return A and the moments to the last accepted epoch, multiply
     the rate by 0.1 and rewind i by tau_f).  The objective is exact (no
     regulariser on s_t, as Algorithm 4 passes mu = 0), the rate and the saved
     copies persist across time steps, and the saved solution starts as the
     initial factors;
  4. the reservoir window update (window.py), storing X_t and s_t (with the
     model-difference history of eq. gcp_stream_problem_2, hist="model",
     only s_t is stored and the gradient is that of model_hist.py);
  5. A_old <- A.
Without epochs (kappa_f = 0) every iteration is kept.

Matrix slices (d = 2, the shape of the paper's first synthetic experiment):
a slice X_t is I1 x I2, the model m_ij = sum_r s_r a_ir b_jr.  It is carried
here as the d = 3 problem with I3 = 1 and a fixed third factor of ones, which
has the same model; only A^(1), A^(2) take ADAM steps and the factor
regulariser covers those two (the fixed row's lam/2 R is left out of F).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from .adam import adam_step
from .gcp import gradient
from .model_hist import gradient_model
from .solve import ls_temporal
from .gcp import objective
from .model_hist import objective_model
from .temporal_sgd import DECAY, temporal_sgd
from .window import window_update


class StreamOracle:
    def __init__(self, A0, X_hist, s_hist, t_hist, *, loss="gaussian",
                 window=0, w=1.0, theta=1.0, lam=0.0, mu=0.0,
                 lower=-np.inf, alpha_f=1e-3, beta1=0.9, beta2=0.999,
                 adam_eps=1e-8, tau_f=1, seed=0, hist="slices", tsolve="ls",
                 tau_w=100, kappa_w=20, alpha_w=1.0, tol_w=-np.inf, kappa_f=0, tol_f=-np.inf, d=3):
        self.d = d
        if d == 2:
            R = np.asarray(A0[0]).shape[1]
            A0 = [A0[0], A0[1], np.ones((1, R))]
            X_hist = [np.asarray(x).reshape(np.asarray(x).shape[:2] + (1,)) for x in X_hist]
        self.A = [np.array(a, np.float64) for a in A0]
        self.A_old = [a.copy() for a in self.A]
        self.u = [np.zeros_like(a) for a in self.A]
        self.v = [np.zeros_like(a) for a in self.A]
        self.i = 0
        self.alpha_f = alpha_f
        self.A_o = [a.copy() for a in self.A]
        self.u_o = [np.zeros_like(a) for a in self.A]
        self.v_o = [np.zeros_like(a) for a in self.A]
        self.slots = [int(t) for t in t_hist]
        self.hist = hist
        self.Xw = [np.array(x, np.float64) for x in X_hist] if hist == "slices" else []
        self.Sw = ([np.array(s, np.float64) for s in np.asarray(s_hist).reshape(len(self.slots), -1)]
                   if self.slots else [])
        self.t = (max(self.slots) + 1) if self.slots else 1
        self.cfg = SimpleNamespace(loss=loss, H=window, w=w, theta=theta,
                                   lam=lam, mu=mu, lower=lower,
                                   alpha_f=alpha_f, beta1=beta1, beta2=beta2,
                                   eps=adam_eps, tau_f=tau_f, seed=seed, tsolve=tsolve,
                                   tau_w=tau_w, kappa_w=kappa_w, alpha_w=alpha_w, tol_w=tol_w,
                                   kappa_f=kappa_f, tol_f=tol_f)

    def problem(self, X_t, s_t, A=None):
        c = self.cfg
        return SimpleNamespace(X_t=X_t, A=self.A if A is None else A, s_t=s_t,
                               A_old=self.A_old, X_hist=self.Xw,
                               s_hist=(np.array(self.Sw).reshape(len(self.Sw), -1) if self.Sw
                                       else np.zeros((0, self.A[0].shape[1]))),
                               t_hist=np.array(self.slots, np.int64), t=self.t,
                               w=c.w, theta=c.theta, lam=c.lam, mu=c.mu,
                               loss=c.loss)

    def solve_st(self, X_t):
        c = self.cfg
        X_t = self._slice3(X_t)
        if c.tsolve == "sgd":
            s, self.solve_info = temporal_sgd(X_t, self.A, c.loss, mu=c.mu, lower=c.lower, alpha=c.alpha_w,
                                              tau=c.tau_w, kappa=c.kappa_w, tol=c.tol_w, beta1=c.beta1,
                                              beta2=c.beta2, eps=c.eps)
            return s
        if self.cfg.loss != "gaussian":
            raise ValueError("least-squares temporal solve needs the Gaussian loss")
        return ls_temporal(X_t, self.A, self.cfg.mu, self.cfg.lower)

    def factor_objective(self, X_t, s_t) -> float:
        """The objective Algorithm 4 compares: every term but mu/2 ||s_t||^2."""
        prob = self.problem(self._slice3(X_t), s_t)
        prob.mu = 0.0
        F = objective(prob) if self.hist == "slices" else objective_model(prob)
        return F - (0.5 * self.cfg.lam * self.A[2].size if self.d == 2 else 0.0)

    def _slice3(self, X_t):
        X_t = np.asarray(X_t, np.float64)
        return X_t.reshape(X_t.shape[:2] + (1,)) if self.d == 2 else X_t

    def _iterations(self, X_t, s_t, n):
        c = self.cfg
        for _ in range(n):
            prob = self.problem(X_t, s_t)
            G, _ = gradient(prob) if self.hist == "slices" else gradient_model(prob)
            for k in range(self.d):
                self.A[k], self.u[k], self.v[k] = adam_step(
                    self.A[k], G[k], self.u[k], self.v[k], self.i, self.alpha_f,
                    c.beta1, c.beta2, c.eps, c.lower)
            self.i += 1

    def update_factors(self, X_t, s_t):
        c = self.cfg
        X_t = self._slice3(X_t)
        if c.kappa_f == 0:
            self._iterations(X_t, s_t, c.tau_f)
        else:
            F = self.factor_objective(X_t, s_t)
            info = SimpleNamespace(F=[F], F_try=[], rolled=[])
            for _ in range(c.kappa_f):
                if not F > c.tol_f:
                    break
                F_old = F
                self._iterations(X_t, s_t, c.tau_f)
                F = self.factor_objective(X_t, s_t)
                info.F_try.append(F)
                if F > F_old:
                    self.A = [a.copy() for a in self.A_o]
                    self.u = [a.copy() for a in self.u_o]
                    self.v = [a.copy() for a in self.v_o]
                    self.alpha_f *= DECAY
                    self.i -= c.tau_f
                    F = F_old
                    info.rolled.append(True)
                else:
                    self.A_o = [a.copy() for a in self.A]
                    self.u_o = [a.copy() for a in self.u]
                    self.v_o = [a.copy() for a in self.v]
                    info.rolled.append(False)
                info.F.append(F)
            self.fac_info = info
        new_slots, slot = window_update(self.slots, c.H, self.t, c.seed)
        if slot >= 0:
            keep = self.hist == "slices"
            if slot == len(self.Sw):
                if keep:
                    self.Xw.append(np.array(X_t, np.float64))
                self.Sw.append(np.array(s_t, np.float64))
            else:
                if keep:
                    self.Xw[slot] = np.array(X_t, np.float64)
                self.Sw[slot] = np.array(s_t, np.float64)
        self.slots = new_slots
        self.A_old = [a.copy() for a in self.A]
        self.t += 1
        return slot

    def step(self, X_t):
        self.A = [a.copy() for a in self.A_old]
        s_t = self.solve_st(X_t)
        self.update_factors(X_t, s_t)
        return s_t
