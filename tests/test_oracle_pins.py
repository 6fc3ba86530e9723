"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, library routines, brute force, invariants).
CPU only."""
import math
from types import SimpleNamespace

import numpy as np
import pytest
from scipy import stats
from scipy.special import gammaln

import gcp_inputs as gi
from oracle import gcp as og
from oracle.adam import adam_step
from oracle.solve import ls_temporal
from oracle.window import splitmix64, window_update, reservoir_draw

LOSSES = og.LOSSES


def tiny(loss, seed=0, dims=(3, 4, 5), R=2, H=2, **kw):
    return gi.random_dense(dims, R, H, loss, seed, dtype=np.float64, **kw)


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ----------------------------------------------------------- losses ----
@pytest.mark.parametrize("loss", LOSSES)
def test_loss_is_negative_log_likelihood(loss):
    """f = -log p(x | l^-1(m)) up to terms free of m (Section 2.2), checked
    against scipy's distributions."""
    g = np.random.default_rng(1)
    m = g.uniform(-2, 2, size=50)
    if loss == "gaussian":
        x = g.normal(size=50)
        # (x-m)^2 = -log N(x; m, sigma^2=1/2) - 0.5 log(pi)
        ref = -stats.norm.logpdf(x, loc=m, scale=math.sqrt(0.5)) - 0.5 * math.log(math.pi)
    elif loss == "poisson_log":
        x = g.poisson(2.0, size=50).astype(float)
        ref = -stats.poisson.logpmf(x, np.exp(m)) - gammaln(x + 1)
    else:
        x = (g.random(50) < 0.4).astype(float)
        ref = -stats.bernoulli.logpmf(x, 1 / (1 + np.exp(-m)))
    np.testing.assert_allclose(og.loss_f(loss, x, m), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("loss", LOSSES)
def test_loss_derivative_central_difference(loss):
    g = np.random.default_rng(2)
    m = g.uniform(-3, 3, size=40)
    x = {"gaussian": g.normal(size=40),
         "poisson_log": g.poisson(1.5, size=40).astype(float),
         "bernoulli_logit": (g.random(40) < 0.5).astype(float)}[loss]
    hstep = 1e-6
    fd = (og.loss_f(loss, x, m + hstep) - og.loss_f(loss, x, m - hstep)) / (2 * hstep)
    np.testing.assert_allclose(og.loss_dfdm(loss, x, m), fd, rtol=1e-7, atol=1e-8)


def test_loss_special_values():
    # Poisson-log: y = 0 where m = log x; Bernoulli-logit at m = 0: f = log 2
    x = np.array([1.0, 2.0, 7.0])
    np.testing.assert_allclose(og.loss_dfdm("poisson_log", x, np.log(x)), 0, atol=1e-14)
    np.testing.assert_allclose(og.loss_f("bernoulli_logit", 0.0, 0.0), math.log(2))
    m = np.linspace(-40, 40, 81)
    for xv in (0.0, 1.0):
        y = og.loss_dfdm("bernoulli_logit", xv, m)
        assert np.all(np.abs(y) <= 1) and np.all(og.loss_f("bernoulli_logit", xv, m) >= 0)
    # stable at large |m|
    assert np.isfinite(og.loss_f("bernoulli_logit", 1.0, 800.0))


# ------------------------------------------------- tensor algebra ------
def test_unfold_and_khatri_rao_definitions():
    """X_(k)[i_k, j] with j running lowest-mode-fastest; Z row order the
    same, so that X_(k) Z_k is the MTTKRP sum over the other indices."""
    g = np.random.default_rng(3)
    X = g.normal(size=(2, 3, 4))
    U = og.unfold(X, 1)
    assert U.shape == (3, 8)
    for i1 in range(2):
        for i2 in range(3):
            for i3 in range(4):
                assert U[i2, i1 + 2 * i3] == X[i1, i2, i3]
    A = [g.normal(size=(n, 2)) for n in (2, 3, 4)]
    Z1 = og.z_except(A, 1)   # A3 (.) A1
    for i1 in range(2):
        for i3 in range(4):
            np.testing.assert_allclose(Z1[i1 + 2 * i3], A[2][i3] * A[0][i1])
    np.testing.assert_allclose(og.full_model(A, np.ones(2)),
                               np.einsum("ir,jr,kr->ijk", *A))


# --------------------------------------------- brute force (tier L) ----
@pytest.mark.parametrize("loss", LOSSES)
def test_tier_v_matches_loops(loss):
    p = tiny(loss, seed=4, theta=0.7, w=1.3, lam=0.1, mu=0.2)
    F = og.objective(p)
    assert abs(F - og.objective_loops(p)) <= 1e-12 * og.loss_terms_abs(p)
    G, gs = og.gradient(p)
    GL, gsL = og.gradient_loops(p)
    for k in range(3):
        assert rel(G[k], GL[k]) < 1e-12
    assert rel(gs, gsL) < 1e-12


# ------------------------------------------------ finite differences ----
@pytest.mark.parametrize("loss", LOSSES)
def test_gradient_matches_central_differences(loss):
    p = tiny(loss, seed=5, dims=(3, 4, 3), R=3, H=2, theta=0.8, w=0.7, lam=0.05, mu=0.3)
    G, gs = og.gradient(p)
    for k in range(3):
        for (r, j) in [(0, 0), (1, 2), (p.dims[k] - 1, 1)]:
            a0 = p.A[k][r, j]
            h = 1e-6 * max(1.0, abs(a0))
            p.A[k][r, j] = a0 + h
            Fp = og.objective(p)
            p.A[k][r, j] = a0 - h
            Fm = og.objective(p)
            p.A[k][r, j] = a0
            fd = (Fp - Fm) / (2 * h)
            assert abs(fd - G[k][r, j]) <= 1e-6 * max(1.0, abs(G[k][r, j])), (k, r, j)
    for j in range(3):
        s0 = p.s_t[j]
        h = 1e-6
        p.s_t[j] = s0 + h
        Fp = og.objective(p)
        p.s_t[j] = s0 - h
        Fm = og.objective(p)
        p.s_t[j] = s0
        assert abs((Fp - Fm) / (2 * h) - gs[j]) <= 1e-6 * max(1.0, abs(gs[j]))


# ---------------------------------------------- Gaussian identity ------
def test_gaussian_gradient_equals_cp_least_squares_gradient():
    """Section 5: for f = (x-m)^2,
    dF/dA^(k) = 2 (A^(k) diag(s) Gamma_k diag(s) - X_(k) Z_k diag(s)) per
    slice (the sign printed in the paper is flipped), with
    Gamma_k = hadamard_{l != k} A^(l)^T A^(l);  dF/ds = 2 (Gamma s - Z^T x).
    Never evaluates the model entrywise."""
    p = tiny("gaussian", seed=6, dims=(4, 5, 6), R=3, H=3, theta=0.9, w=1.1, lam=0.2, mu=0.4)
    G, gs = og.gradient(p)
    A = p.A
    grams = [a.T @ a for a in A]
    slices = [(p.X_t, p.s_t, 1.0)] + [
        (p.X_hist[h], p.s_hist[h], p.w * p.theta ** (p.t - p.t_hist[h])) for h in range(3)]
    for k in range(3):
        Gk = np.prod([grams[l] for l in range(3) if l != k], axis=0)
        ref = p.lam * A[k]
        for X, s, c in slices:
            B = np.einsum("ijk,jr,kr->ir", *((X,) + tuple(A[l] for l in range(3) if l != k))) \
                if k == 0 else None
            # MTTKRP of X by an independent einsum per mode
            sub = {0: "ijk,jr,kr->ir", 1: "ijk,ir,kr->jr", 2: "ijk,ir,jr->kr"}[k]
            B = np.einsum(sub, X, *[A[l] for l in range(3) if l != k])
            ref = ref + c * 2 * (A[k] @ np.diag(s) @ Gk @ np.diag(s) - B @ np.diag(s))
        assert rel(G[k], ref) < 1e-12
    Gam = np.prod(grams, axis=0)
    b = np.einsum("ijk,ir,jr,kr->r", p.X_t, *A)
    assert rel(gs, 2 * (Gam @ p.s_t - b) + p.mu * p.s_t) < 1e-12


# ---------------------------------------------------- closed forms -----
def test_zero_weights_closed_forms():
    """s_t = 0, no window: m = 0 everywhere."""
    g = np.random.default_rng(7)
    dims = (3, 4, 5)
    A = [g.normal(size=(n, 3)) for n in dims]
    X = g.poisson(1.0, size=dims).astype(float)
    omega = np.prod(dims)
    colsum = np.prod([a.sum(axis=0) for a in A], axis=0)
    b = np.einsum("ijk,ir,jr,kr->r", X, *A)
    for loss, F0, gs0 in [
        ("gaussian", np.sum(X ** 2), -2 * b),
        ("poisson_log", omega, colsum - b),
        ("bernoulli_logit", omega * math.log(2), 0.5 * colsum - b),
    ]:
        Xl = (X > 0).astype(float) if loss == "bernoulli_logit" else X
        if loss == "bernoulli_logit":
            b2 = np.einsum("ijk,ir,jr,kr->r", Xl, *A)
            gs0 = 0.5 * colsum - b2
        p = SimpleNamespace(X_t=Xl, A=A, s_t=np.zeros(3), X_hist=[], s_hist=np.zeros((0, 3)),
                            t_hist=np.zeros(0, np.int64), t=1, w=1.0, theta=1.0,
                            lam=0.3, mu=0.5, loss=loss)
        F = og.objective(p)
        assert abs(F - (F0 + 0.15 * sum(np.sum(a * a) for a in A))) < 1e-9 * max(1, abs(F0))
        G, gs = og.gradient(p)
        for k in range(3):
            assert rel(G[k], 0.3 * A[k]) < 1e-13
        assert rel(gs, gs0) < 1e-12


def test_noiseless_planted_gaussian_is_stationary():
    g = np.random.default_rng(8)
    dims = (4, 5, 6)
    A = [g.normal(size=(n, 3)) for n in dims]
    S = g.uniform(0.5, 1.5, size=(4, 3))
    Xs = [og.full_model(A, S[h]) for h in range(4)]
    p = SimpleNamespace(X_t=Xs[3], A=A, s_t=S[3], X_hist=Xs[:3], s_hist=S[:3],
                        t_hist=np.arange(1, 4), t=4, w=1.0, theta=0.9, lam=0.0,
                        mu=0.0, loss="gaussian")
    assert og.objective(p) < 1e-20
    G, gs = og.gradient(p)
    assert max(np.abs(x).max() for x in G + [gs]) < 1e-11
    np.testing.assert_allclose(ls_temporal(Xs[3], A), S[3], rtol=1e-10)


# ------------------------------------------------------ invariants -----
@pytest.mark.parametrize("loss", LOSSES)
def test_column_scaling_invariance(loss):
    p = tiny(loss, seed=9, R=3, H=2)
    F = og.objective(p)
    G, gs = og.gradient(p)
    c = 1.7
    p.A[0][:, 1] *= c
    p.A[1][:, 1] /= c
    F2 = og.objective(p)
    G2, gs2 = og.gradient(p)
    assert abs(F - F2) < 1e-12 * og.loss_terms_abs(p)
    np.testing.assert_allclose(G2[0][:, 1], G[0][:, 1] / c, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(G2[1][:, 1], G[1][:, 1] * c, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(G2[2], G[2], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gs2, gs, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("loss", LOSSES)
def test_mode_permutation(loss):
    p = tiny(loss, seed=10, dims=(3, 4, 5), R=2, H=1)
    G, gs = og.gradient(p)
    perm = (2, 0, 1)
    q = SimpleNamespace(**vars(p))
    q.X_t = np.transpose(p.X_t, perm)
    q.X_hist = [np.transpose(x, perm) for x in p.X_hist]
    q.A = [p.A[k] for k in perm]
    Gq, gsq = og.gradient(q)
    for n, k in enumerate(perm):
        assert rel(Gq[n], G[k]) < 1e-12
    assert rel(gsq, gs) < 1e-12


@pytest.mark.parametrize("loss", LOSSES)
def test_window_term_is_additive(loss):
    """Duplicating a stored slice doubles its contribution; weight w=0
    reduces eq. gcp_stream_problem_1 to eq. gcp_stream_t."""
    p = tiny(loss, seed=11, H=1)
    q = SimpleNamespace(**vars(p))
    q.X_hist, q.s_hist, q.t_hist = [], np.zeros((0, p.rank)), np.zeros(0, np.int64)
    r = SimpleNamespace(**vars(p))
    r.X_hist = [p.X_hist[0], p.X_hist[0]]
    r.s_hist = np.stack([p.s_hist[0], p.s_hist[0]])
    r.t_hist = np.array([p.t_hist[0]] * 2)
    F0, F1, F2 = og.objective(q), og.objective(p), og.objective(r)
    assert abs((F2 - F0) - 2 * (F1 - F0)) < 1e-12 * og.loss_terms_abs(r)
    (G0, _), (G1, _), (G2, _) = og.gradient(q), og.gradient(p), og.gradient(r)
    for k in range(3):
        assert rel(G2[k] - G0[k], 2 * (G1[k] - G0[k])) < 1e-11
    z = SimpleNamespace(**vars(p))
    z.w = 0.0
    assert abs(og.objective(z) - F0) < 1e-12 * og.loss_terms_abs(p)


def test_history_weight_formula():
    np.testing.assert_allclose(og.history_weights(10, [7, 9], 2.0, 0.5), [2 * 0.125, 2 * 0.5])


# --------------------------------------------------------- LS solve ----
def test_ls_solve_normal_equations_and_library():
    g = np.random.default_rng(12)
    A = [g.normal(size=(n, 4)) for n in (5, 6, 7)]
    X = g.normal(size=(5, 6, 7))
    mu = 0.3
    s = ls_temporal(X, A, mu)
    # residual of the normal equations Z^T (x - Z s) = mu/2 s, with Z formed
    # by an independent einsum
    Z = np.einsum("ir,jr,kr->ijkr", *A).reshape(-1, 4)
    x = X.reshape(-1)
    np.testing.assert_allclose(Z.T @ (x - Z @ s), 0.5 * mu * s, rtol=1e-9, atol=1e-10)
    s0 = ls_temporal(X, A, 0.0)
    np.testing.assert_allclose(s0, np.linalg.lstsq(Z, x, rcond=None)[0], rtol=1e-10)
    # stationarity of the oracle's own temporal gradient at the solution
    p = SimpleNamespace(X_t=X, A=A, s_t=s, X_hist=[], s_hist=np.zeros((0, 4)),
                        t_hist=np.zeros(0, np.int64), t=1, w=1.0, theta=1.0,
                        lam=0.0, mu=mu, loss="gaussian")
    _, gs = og.gradient(p)
    assert np.abs(gs).max() < 1e-9 * np.abs(Z.T @ x).max()
    assert np.all(ls_temporal(X, A, mu, lower=0.0) >= 0)


# ------------------------------------------------------------- Adam ----
def test_adam_closed_form_constant_gradient():
    """With u = v = 0 and a constant gradient g for n steps,
    u_n = (1-b1^n) g, v_n = (1-b2^n) g^2, so each step moves a by
    alpha g / (|g| + eps / sqrt(1 - b2^n))."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    a = np.array([1.0, 2.0, 3.0, 4.0])
    u = np.zeros(4)
    v = np.zeros(4)
    alpha, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    expect = a.copy()
    for i in range(5):
        a, u, v = adam_step(a, g, u, v, i, alpha, b1, b2, eps)
        n = i + 1
        expect = expect - alpha * g / (np.abs(g) + eps / math.sqrt(1 - b2 ** n))
        np.testing.assert_allclose(a, expect, rtol=1e-13, atol=1e-15)
    a2, _, _ = adam_step(np.array([0.01]), np.array([5.0]), np.zeros(1), np.zeros(1), 0,
                         1.0, lower=0.0)
    assert a2[0] == 0.0


# --------------------------------------------------- window / RNG ------
def test_splitmix64_known_outputs():
    """Published SplitMix64 outputs for state 0 (fixtures in
    tests/golden/splitmix64.txt)."""
    import pathlib
    rows = [l.split() for l in (pathlib.Path(__file__).parent / "golden" / "splitmix64.txt")
            .read_text().splitlines() if l and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    for n, hexval in rows:
        assert splitmix64((int(n) * gamma) & ((1 << 64) - 1)) == int(hexval, 16)


def test_window_fills_then_reservoir():
    slots = []
    for t in range(1, 4):
        slots, slot = window_update(slots, 3, t, seed=5)
        assert slot == t - 1
    assert slots == [1, 2, 3]
    for t in range(4, 50):
        before = list(slots)
        slots, slot = window_update(slots, 3, t, seed=5)
        j = reservoir_draw(5, t)
        assert (slot == j - 1) == (j <= 3)
        if slot >= 0:
            assert slots[slot] == t and [x for i, x in enumerate(slots) if i != slot] == \
                [x for i, x in enumerate(before) if i != slot]
        else:
            assert slots == before


def test_reservoir_inclusion_is_uniform():
    """After step T the window is a uniform sample: each past step is kept
    with probability H/T (chi-square over many seeds)."""
    H, T, trials = 4, 30, 4000
    counts = np.zeros(T + 1)
    for seed in range(trials):
        slots = []
        for t in range(1, T + 1):
            slots, _ = window_update(slots, H, t, seed * 7919 + 13)
        for s in slots:
            counts[s] += 1
    obs = counts[1:]
    exp = trials * H / T
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert stats.chi2.sf(chi2, T - 1) > 1e-4, chi2


# ------------------------------------------- identity / odds links ----
@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_paper_link_losses_are_negative_log_likelihoods(loss):
    """Section 2.2's identity-link Poisson and odds-link Bernoulli losses:
    f = -log p(x | l^-1(m)) up to terms free of m (eps = 1e-10 moves f by at
    most x eps / m)."""
    g = np.random.default_rng(11)
    m = g.uniform(0.05, 4.0, size=60)
    if loss == "poisson_id":
        x = g.poisson(2.0, size=60).astype(float)
        nll = -stats.poisson.logpmf(x, m)
        const = gammaln(x + 1.0)
    else:
        x = (g.random(60) < 0.4).astype(float)
        nll = -stats.bernoulli.logpmf(x, m / (1.0 + m))
        const = 0.0
    assert np.allclose(og.loss_f(loss, x, m) + const, nll, rtol=1e-9, atol=1e-8)


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_paper_link_loss_derivatives_are_central_differences(loss):
    g = np.random.default_rng(12)
    m = g.uniform(0.1, 3.0, size=40)
    x = g.poisson(1.5, size=40).astype(float) if loss == "poisson_id" else (g.random(40) < 0.5).astype(float)
    h = 1e-6
    fd = (og.loss_f(loss, x, m + h) - og.loss_f(loss, x, m - h)) / (2 * h)
    assert np.allclose(og.loss_dfdm(loss, x, m), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("loss", og.PAPER_LOSSES)
def test_paper_link_gradient_matches_brute_force_loops(loss):
    """The matrix formulas of the gradient with these losses agree with the
    index-by-index loops on a tiny nonnegative instance."""
    p = gi.nonneg_dense((3, 4, 5), 2, 2, loss, seed=13, lam=0.1, mu=0.2, dtype=np.float64)
    assert og.objective(p) == pytest.approx(og.objective_loops(p), rel=1e-12)
    G, gs = og.gradient(p)
    Gl, gsl = og.gradient_loops(p)
    for k in range(3):
        assert rel(G[k], Gl[k]) <= 1e-12
    assert rel(gs, gsl) <= 1e-12
