"""End-to-end pins of the oracle's OnlineGCP stream (Algorithm 1 composed of
the temporal solve, the factor iterations or epochs, the reservoir window and
the A_old copy) by recovery of a planted K-tensor.

The paper prints no numbers for its stream experiments (the figures of
Section 6 are absent), so the composition is pinned by what the data's
construction fixes instead:

* C1 (Gaussian, 20x30x40, rank 4, window 3): every slice is the planted
  model plus noise whose Frobenius norm is 10% of the model's, so a model
  that has recovered the planted factors has the local loss of eq.
  `local_loss` of the planted model itself, ||N_t||^2 / ||X_t||^2, which is
  close to 0.1^2 / (1 + 0.1^2) = 0.0099.  A fitted rank-4 model can absorb
  a little of the noise but not much (a few hundred parameters against
  24,000 entries), so the ratio to that floor must end in a narrow band.
* A small Poisson count stream with the log link (planted log-rate
  K-tensor), temporal weights from Algorithm 3 and factor epochs of
  Algorithm 4: the deviance (loss minus the loss of the saturated model
  m = log x) of the fitted model must come down to that of the planted
  model.
* In both, the K-tensor score of Section 6.1 against the planted K-tensor
  must rise from the perturbed start's value to a threshold.  The thresholds
  were set once from the oracle's own run (C1: every late step at 0.997 or
  more; Poisson: 0.93 or more after the first step) with a margin, and are
  fixed here.

A sign error in any gradient term, a wrong ADAM step or bias correction, a
wrong temporal solve, the window weights applied to the wrong slices or a
stale A_old each keep the local loss well above the floor or the score
below its threshold (the last three tests plant such mistakes in copies of
the oracle's pieces and check that the pins catch them).
"""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle.metrics import ktensor_score, local_loss, slice_loss
from oracle.solve import ls_temporal
from oracle.stream import StreamOracle
from oracle.temporal_sgd import temporal_sgd

C1_H = 3


def c1_start(seed=7):
    """C1 data, a perturbed planted start A_true + 0.1 N(0,1), and warm-start
    weights of the first H slices from the least-squares solve at that start."""
    data = gi.c1_stream()
    g = gi.rng(seed)
    A0 = [a + 0.1 * g.standard_normal(a.shape) for a in data.A_true]
    S0 = np.array([ls_temporal(data.X[h], A0, 0.0, -np.inf) for h in range(C1_H)])
    return data, A0, S0


def noise_floor(data, t):
    """Local loss of the planted model on slice t: ||X_t - M_t||^2 / ||X_t||^2."""
    M = gi.ktensor_full(data.A_true, data.S_true[t])
    return float(np.sum((data.X[t] - M) ** 2) / np.sum(data.X[t] ** 2))


def run_c1(alpha_f=1e-2, tau_f=20, oracle_cls=StreamOracle):
    data, A0, S0 = c1_start()
    orc = oracle_cls(A0, [data.X[h] for h in range(C1_H)], S0, np.arange(1, C1_H + 1), loss="gaussian",
                     window=C1_H, alpha_f=alpha_f, tau_f=tau_f, seed=0)
    ratios, scores = [], []
    for t in range(C1_H, data.X.shape[0]):
        s = orc.step(data.X[t])
        ratios.append(local_loss(data.X[t], orc.A, s, "gaussian") / noise_floor(data, t))
        scores.append(ktensor_score(orc.A, s, data.A_true, data.S_true[t]))
    return data, A0, np.array(ratios), np.array(scores)


def test_c1_noise_floor_is_about_one_percent():
    data = gi.c1_stream()
    for t in range(data.X.shape[0]):
        assert abs(noise_floor(data, t) - 0.01 / 1.01) < 1.5e-3


def test_c1_stream_recovers_planted_factors():
    data, A0, ratios, scores = run_c1()
    s0 = ls_temporal(data.X[C1_H], A0, 0.0, -np.inf)
    start_ratio = local_loss(data.X[C1_H], A0, s0, "gaussian") / noise_floor(data, C1_H)
    start_score = ktensor_score(A0, s0, data.A_true, data.S_true[C1_H])
    assert start_ratio > 3.0 and start_score < 0.985        # the start is clearly off
    assert np.all(ratios[4:] <= 1.01) and np.all(ratios[4:] >= 0.97), ratios
    assert np.all(scores[4:] >= 0.997), scores
    # the paper's C1 rate (alpha_f = 1e-3, tau_f = 100) converges too, a little later
    _, _, ratios2, scores2 = run_c1(alpha_f=1e-3, tau_f=100)
    assert np.all(ratios2[6:] <= 1.01) and np.all(scores2[6:] >= 0.997)


def deviance(X, A, s):
    """Poisson-log loss minus that of the saturated model (m = log x)."""
    f, _ = slice_loss(X, A, s, "poisson_log")
    pos = X > 0
    sat = float(np.sum(X) - np.sum(X[pos] * np.log(X[pos])))
    return f - sat


POIS_H = 3


def poisson_start(seed=22):
    data = gi.poisson_log_stream()
    g = gi.rng(seed)
    A0 = [a + 0.3 * g.standard_normal(a.shape) for a in data.A_true]
    sgd = lambda X, A: temporal_sgd(X, A, "poisson_log", mu=0.0, lower=-np.inf, alpha=1.0, tau=100,
                                    kappa=20, tol=-np.inf, beta1=0.9, beta2=0.999, eps=1e-8)[0]
    S0 = np.array([sgd(data.X[h], A0) for h in range(POIS_H)])
    return data, A0, S0, sgd


def test_poisson_stream_with_weight_sgd_and_epochs_recovers_planted_factors():
    data, A0, S0, sgd = poisson_start()
    orc = StreamOracle(A0, [data.X[h] for h in range(POIS_H)], S0, np.arange(1, POIS_H + 1),
                       loss="poisson_log", window=POIS_H, alpha_f=1e-2, tau_f=20, kappa_f=5, seed=3,
                       tsolve="sgd", tau_w=100, kappa_w=20, alpha_w=1.0)
    s0 = sgd(data.X[POIS_H], A0)
    d_true = deviance(data.X[POIS_H], data.A_true, data.S_true[POIS_H])
    assert deviance(data.X[POIS_H], A0, s0) / d_true > 1.05
    assert ktensor_score(A0, s0, data.A_true, data.S_true[POIS_H]) < 0.6
    dev, sc = [], []
    for t in range(POIS_H, data.X.shape[0]):
        s = orc.step(data.X[t])
        dev.append(deviance(data.X[t], orc.A, s) / deviance(data.X[t], data.A_true, data.S_true[t]))
        sc.append(ktensor_score(orc.A, s, data.A_true, data.S_true[t]))
    dev, sc = np.array(dev), np.array(sc)
    assert np.all(dev[1:] <= 1.0) and np.all(dev[1:] >= 0.97), dev
    assert np.all(sc[1:] >= 0.92), sc


# ---- the pins catch planted mistakes ----------------------------------------

class _StaleAold(StreamOracle):
    """Mistake: the factors of a step start from A0 forever (A_old never copied)."""

    def update_factors(self, X_t, s_t):
        keep = [a.copy() for a in self.A_old]
        slot = super().update_factors(X_t, s_t)
        self.A_old = keep
        return slot


class _FlippedWindow(StreamOracle):
    """Mistake: the window term enters the objective with the wrong sign."""

    def problem(self, X_t, s_t, A=None):
        p = super().problem(X_t, s_t, A)
        p.w = -abs(p.w)
        return p


def test_pin_catches_stale_factor_copy():
    _, _, ratios, scores = run_c1(oracle_cls=_StaleAold)
    assert not (np.all(ratios[4:] <= 1.01) and np.all(scores[4:] >= 0.997))


def test_pin_catches_flipped_window_sign():
    _, _, ratios, scores = run_c1(oracle_cls=_FlippedWindow)
    assert not (np.all(ratios[4:] <= 1.01) and np.all(scores[4:] >= 0.997))


def test_pin_catches_wrong_gradient_sign(monkeypatch):
    import oracle.stream as osm
    real = osm.gradient

    def flipped(prob):
        G, gs = real(prob)
        return [-g for g in G], gs
    monkeypatch.setattr(osm, "gradient", flipped)
    _, _, ratios, scores = run_c1()
    assert not (np.all(ratios[4:] <= 1.01) and np.all(scores[4:] >= 0.997))
