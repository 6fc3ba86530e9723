"""Pins of the metric oracle (Section 6): closed forms, invariances and a
brute-force matching."""
import itertools

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import metrics as om


def test_local_loss_closed_forms():
    g = np.random.default_rng(0)
    X = g.normal(size=(4, 5, 6))
    A = [g.normal(size=(n, 3)) for n in X.shape]
    # Gaussian, zero model: sum x^2 / ||X||^2 = 1
    assert om.local_loss(X, A, np.zeros(3), "gaussian") == pytest.approx(1.0, rel=1e-15)
    # Gaussian, exact model: 0
    s = g.uniform(0.5, 1.5, 3)
    M = np.einsum("ir,jr,kr,r->ijk", *A, s)
    assert om.local_loss(M, A, s, "gaussian") == pytest.approx(0.0, abs=1e-20)
    # Poisson-log at m = 0: every entry costs exp(0) = 1
    C = g.poisson(2.0, size=(4, 5, 6)).astype(float)
    assert om.local_loss(C, A, np.zeros(3), "poisson_log") == pytest.approx(C.size / np.sum(C * C), rel=1e-15)
    # Bernoulli-logit at m = 0: log 2 per entry
    Bx = (g.random((4, 5, 6)) < 0.4).astype(float)
    assert om.local_loss(Bx, A, np.zeros(3), "bernoulli_logit") == pytest.approx(
        Bx.size * np.log(2.0) / np.sum(Bx), rel=1e-14)


def test_global_loss_is_the_stacked_ratio():
    g = np.random.default_rng(1)
    Xs = [g.normal(size=(3, 4, 5)) for _ in range(3)]
    A = [g.normal(size=(n, 2)) for n in (3, 4, 5)]
    S = [g.uniform(size=2) for _ in range(3)]
    num = sum(np.sum((X - np.einsum("ir,jr,kr,r->ijk", *A, s)) ** 2) for X, s in zip(Xs, S))
    den = sum(np.sum(X ** 2) for X in Xs)
    assert om.global_loss(Xs, A, S, "gaussian") == pytest.approx(num / den, rel=1e-14)


def test_score_is_one_for_the_same_ktensor_up_to_scaling_and_order():
    g = np.random.default_rng(2)
    B = [g.normal(size=(n, 4)) for n in (6, 7, 8)]
    wb = g.uniform(1, 2, 4)
    assert om.ktensor_score(B, wb, B, wb) == pytest.approx(1.0, rel=1e-14)
    perm = [2, 0, 3, 1]
    c = [g.uniform(0.5, 2, 4) for _ in range(3)]
    A = [b[:, perm] * ck for b, ck in zip(B, c)]
    wa = wb[perm] / (c[0] * c[1] * c[2])
    assert om.ktensor_score(A, wa, B, wb) == pytest.approx(1.0, rel=1e-12)
    # a sign flip in two modes leaves the K-tensor unchanged
    A2 = [B[0] * -1, B[1] * -1, B[2]]
    assert om.ktensor_score(A2, wb, B, wb) == pytest.approx(1.0, rel=1e-12)


def test_score_penalises_weights_and_noise():
    g = np.random.default_rng(3)
    B = [g.normal(size=(n, 3)) for n in (5, 6, 7)]
    wb = np.ones(3)
    assert om.ktensor_score(B, 2 * wb, B, wb) == pytest.approx(0.5, rel=1e-12)
    noisy = [b + 0.3 * g.normal(size=b.shape) for b in B]
    s1 = om.ktensor_score(noisy, wb, B, wb)
    noisier = [b + 1.0 * g.normal(size=b.shape) for b in B]
    assert 0 < om.ktensor_score(noisier, wb, B, wb) < s1 < 1


def test_greedy_matching_equals_brute_force_on_separated_components():
    g = np.random.default_rng(4)
    B = [np.linalg.qr(g.normal(size=(9, 4)))[0] for _ in range(3)]
    wb = g.uniform(1, 2, 4)
    A = [b + 0.05 * g.normal(size=b.shape) for b in B]
    perm = [3, 1, 0, 2]
    A = [a[:, perm] for a in A]
    wa = wb[perm] * g.uniform(0.9, 1.1, 4)
    P = om.pair_scores(A, wa, B, wb)
    best = max(sum(P[i, p[i]] for i in range(4)) for p in itertools.permutations(range(4))) / 4
    assert om.ktensor_score(A, wa, B, wb) == pytest.approx(best, rel=1e-14)
