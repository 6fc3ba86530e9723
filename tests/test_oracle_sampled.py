"""Pins of the sampled-gradient oracle (Section 4.3, Algorithm 6): the
counter-based generator against its published outputs, the stratified
sampler's invariants and statistics, and unbiasedness against the dense
oracle.  CPU only."""
import pathlib
from types import SimpleNamespace

import numpy as np
import pytest
from scipy import stats

import gcp_inputs as gi
from oracle import gcp as og
from oracle import sampled as osm

GOLDEN = pathlib.Path(__file__).parent / "golden"


def test_philox_known_answers():
    for line in (GOLDEN / "philox4x32_10.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        out = osm.philox4x32_10([[v[0]], [v[1]], [v[2]], [v[3]]], (v[4], v[5]))
        assert [int(o[0]) for o in out] == v[6:]


def _small_sparse(seed=1, dims=(6, 7, 8), nnz=100, window=2, p=40, q=60, loss="poisson_log"):
    return gi.sparse_problem(dims=dims, rank=3, window=window, nnz=nnz, p=p, q=q, seed=seed,
                             loss=loss)


def test_zero_draws_never_hit_nonzeros_and_are_uniform():
    prob = _small_sparse(nnz=120, q=20000)
    coo = prob.X_t
    lin = (coo.coords[:, 0].astype(np.int64) * 7 + coo.coords[:, 1]) * 8 + coo.coords[:, 2]
    z, att = osm.draw_zeros(prob.seed, prob.t, 0, prob.q, coo.dims, lin)
    zl = (z[:, 0] * 7 + z[:, 1]) * 8 + z[:, 2]
    assert not np.isin(zl, lin).any()
    assert att.max() >= 1              # rejections happened (density ~36%)
    # each zero cell equally likely: chi-square over the zero cells
    zeros = np.setdiff1d(np.arange(6 * 7 * 8), lin)
    counts = np.bincount(zl, minlength=6 * 7 * 8)[zeros]
    chi2 = float(np.sum((counts - counts.mean()) ** 2 / counts.mean()))
    assert stats.chi2.sf(chi2, zeros.size - 1) > 1e-4


def test_nonzero_draws_uniform_over_stored_entries():
    idx = osm.draw_nonzeros(seed=3, stamp=5, call=2, p=50000, eta=37)
    assert idx.min() >= 0 and idx.max() < 37
    counts = np.bincount(idx, minlength=37)
    chi2 = float(np.sum((counts - counts.mean()) ** 2 / counts.mean()))
    assert stats.chi2.sf(chi2, 36) > 1e-4


def _dense_equivalent(prob):
    def dense(coo):
        X = np.zeros(coo.dims)
        X[tuple(coo.coords.T)] = coo.vals
        return X
    return SimpleNamespace(X_t=dense(prob.X_t), A=prob.A, s_t=prob.s_t,
                           X_hist=[dense(x) for x in prob.X_hist], s_hist=prob.s_hist,
                           t_hist=prob.t_hist, t=prob.t, w=prob.w, theta=prob.theta,
                           lam=prob.lam, mu=prob.mu, loss=prob.loss)


@pytest.mark.parametrize("loss", ["poisson_log", "bernoulli_logit"])
def test_sampled_gradient_is_unbiased(loss):
    """E[ytilde] = y (Section 4.3): the mean of many independent sampled
    gradients (different call numbers) approaches the exact gradient of the
    dense oracle within CLT bands."""
    prob = _small_sparse(nnz=80, p=30, q=40, loss=loss)
    prob.lam, prob.mu, prob.theta, prob.w = 0.1, 0.2, 0.8, 1.5
    K = 600
    draws = [osm.sampled_loss_grad(prob, call=c) for c in range(K)]
    Gex, gsex = og.gradient(_dense_equivalent(prob))
    Fex = og.objective(_dense_equivalent(prob))
    for k in range(3):
        samp = np.stack([d[1][k] for d in draws])
        mean, se = samp.mean(0), samp.std(0, ddof=1) / np.sqrt(K)
        z = np.abs(mean - Gex[k]) / np.maximum(se, 1e-12)
        assert np.mean(z < 4.0) > 0.98 and z.max() < 6.5, z.max()
    samp = np.stack([d[2] for d in draws])
    z = np.abs(samp.mean(0) - gsex) / (samp.std(0, ddof=1) / np.sqrt(K))
    assert z.max() < 6.0
    Fs = np.array([d[0] for d in draws])
    assert abs(Fs.mean() - Fex) < 5 * Fs.std(ddof=1) / np.sqrt(K)


def test_sampled_equals_dense_formula_on_its_own_draws():
    """For a fixed draw list the estimate is the MTTKRP of ytilde: recompute
    it with an independent scatter (einsum per draw)."""
    prob = _small_sparse(nnz=50, p=7, q=5, window=1)
    F, G, g_s = osm.sampled_loss_grad(prob, call=3)
    Gr = [prob.lam * a.copy() for a in prob.A]
    gsr = prob.mu * prob.s_t.copy()
    slices = [(prob.X_t, prob.s_t, 1.0, prob.t),
              (prob.X_hist[0], prob.s_hist[0], prob.w * prob.theta ** (prob.t - prob.t_hist[0]),
               int(prob.t_hist[0]))]
    for n, (coo, s, c, stamp) in enumerate(slices):
        coords, x, wgt = osm.sampled_terms(prob.loss, coo, s, prob.A, prob.seed, stamp, 3,
                                           prob.p, prob.q)
        for (i1, i2, i3), xv, wv in zip(coords, x, wgt):
            m = float(np.einsum("r,r,r,r->", s, prob.A[0][i1], prob.A[1][i2], prob.A[2][i3]))
            y = c * wv * float(og.loss_dfdm(prob.loss, xv, m))
            Gr[0][i1] += y * s * prob.A[1][i2] * prob.A[2][i3]
            Gr[1][i2] += y * s * prob.A[0][i1] * prob.A[2][i3]
            Gr[2][i3] += y * s * prob.A[0][i1] * prob.A[1][i2]
            if n == 0:
                gsr += y * prob.A[0][i1] * prob.A[1][i2] * prob.A[2][i3]
    for k in range(3):
        np.testing.assert_allclose(G[k], Gr[k], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g_s, gsr, rtol=1e-12, atol=1e-12)
