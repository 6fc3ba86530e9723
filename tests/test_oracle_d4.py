"""Oracle pins for four-way tensors (d = 4, slices I1 x I2 x I3 x I4): the
objective and gradients against explicit summation over every multi-index
and against central differences, and the identities that the library's
merged-mode evaluation rests on."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og

LOSSES = ["gaussian", "poisson_log", "bernoulli_logit"]


def tiny4(loss, seed, dims=(2, 3, 2, 3), R=2, H=2, **kw):
    return gi.random_dense(dims, R, H, loss, seed, dtype=np.float64, **kw)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("loss", LOSSES)
def test_four_way_matches_loops(loss):
    p = tiny4(loss, seed=7, theta=0.8, w=1.2, lam=0.1, mu=0.2)
    assert p.X_t.ndim == 4 and len(p.A) == 4
    assert abs(og.objective(p) - og.objective_loops(p)) <= 1e-12 * og.loss_terms_abs(p)
    G, gs = og.gradient(p)
    GL, gsL = og.gradient_loops(p)
    for k in range(4):
        assert rel(G[k], GL[k]) < 1e-12, k
    assert rel(gs, gsL) < 1e-12


@pytest.mark.parametrize("loss", LOSSES)
def test_four_way_gradient_matches_central_differences(loss):
    p = tiny4(loss, seed=8, theta=0.9, w=0.7, lam=0.05, mu=0.3)
    G, gs = og.gradient(p)
    h = 1e-6
    for k in range(4):
        for idx in [(0, 0), (p.A[k].shape[0] - 1, 1)]:
            a0 = p.A[k][idx]
            p.A[k][idx] = a0 + h
            fp = og.objective(p)
            p.A[k][idx] = a0 - h
            fm = og.objective(p)
            p.A[k][idx] = a0
            assert (fp - fm) / (2 * h) == pytest.approx(G[k][idx], rel=1e-6, abs=1e-8), (k, idx)
    for j in range(p.rank):
        s0 = p.s_t[j]
        p.s_t[j] = s0 + h
        fp = og.objective(p)
        p.s_t[j] = s0 - h
        fm = og.objective(p)
        p.s_t[j] = s0
        assert (fp - fm) / (2 * h) == pytest.approx(gs[j], rel=1e-6, abs=1e-8), j


def _merged(p):
    """The three-way problem with modes 3 and 4 merged: entry (i3, i4) ->
    row i3 I4 + i4 (the slice's memory unchanged), factor row
    A3[i3] * A4[i4] (a Khatri-Rao row)."""
    I1, I2, I3, I4 = p.X_t.shape
    A34 = (p.A[2][:, None, :] * p.A[3][None, :, :]).reshape(I3 * I4, -1)
    q = gi.DenseProblem((I1, I2, I3 * I4), p.rank, p.loss, p.X_t.reshape(I1, I2, I3 * I4),
                        [p.A[0], p.A[1], A34], p.s_t, [x.reshape(I1, I2, I3 * I4) for x in p.X_hist],
                        p.s_hist, p.t_hist, p.t, p.w, p.theta, p.lam, p.mu, np.float64)
    return q, A34


@pytest.mark.parametrize("loss", LOSSES)
def test_merged_modes_give_the_four_way_objective_and_gradients(loss):
    """Merging modes 3 and 4 changes the model nowhere, so the data terms
    agree; the regulariser differs by lam/2 (||A3||^2 + ||A4||^2 - ||A34||^2);
    G34 projects onto modes 3 and 4 by the chain rule through the
    Khatri-Rao rows: G3[i3] = sum_i4 G34[i3 I4 + i4] * A4[i4] and
    G4[i4] = sum_i3 G34[i3 I4 + i4] * A3[i3] (plus lam A3, lam A4)."""
    p = tiny4(loss, seed=9, dims=(3, 2, 3, 4), R=3, H=2, theta=0.9, w=1.1, lam=0.07, mu=0.2)
    q, A34 = _merged(p)
    I3, I4 = p.A[2].shape[0], p.A[3].shape[0]
    lam = p.lam
    reg_fix = 0.5 * lam * (np.sum(p.A[2] ** 2) + np.sum(p.A[3] ** 2) - np.sum(A34 ** 2))
    assert og.objective(q) + reg_fix == pytest.approx(og.objective(p), rel=1e-12)
    G4w, gs4 = og.gradient(p)
    q.lam = 0.0
    G3w, gs3 = og.gradient(q)
    assert rel(G3w[0] + lam * p.A[0], G4w[0]) < 1e-12
    assert rel(G3w[1] + lam * p.A[1], G4w[1]) < 1e-12
    G34 = G3w[2].reshape(I3, I4, -1)
    G3 = np.einsum("abr,br->ar", G34, p.A[3]) + lam * p.A[2]
    G4 = np.einsum("abr,ar->br", G34, p.A[2]) + lam * p.A[3]
    assert rel(G3, G4w[2]) < 1e-12 and rel(G4, G4w[3]) < 1e-12
    assert rel(gs3, gs4) < 1e-12
