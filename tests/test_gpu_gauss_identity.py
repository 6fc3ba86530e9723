"""Gradient-only Gaussian calls through the identity of Section 5 (flag
GCP_FLAG_GAUSS_IDENTITY): a data pass without the model plus FP64 Gram
terms, against the oracle's gradient and stream."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import model_hist as omh
from oracle.stream import StreamOracle

from helpers import TOL, make_stream, grad_err, rel_err, to_device

pytestmark = pytest.mark.gpu

SHAPES = [((5, 6, 7), 4, 0), ((7, 9, 70), 5, 2), ((17, 33, 129), 16, 3), ((9, 4, 64), 32, 1),
          ((6, 5, 200), 16, 20), ((3, 3, 3), 64, 1)]


def _grad(prob, **kw):
    import torch
    dev = to_device(prob)
    st = make_stream(prob, dev, gauss_identity=True, **kw)
    _, G, gs = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], want_loss=False)
    torch.cuda.synchronize()
    assert st.sync() == 0
    return [g.double().cpu().numpy() for g in G], gs.double().cpu().numpy()


@pytest.mark.parametrize("kernel", ["valu", "mfma"])
@pytest.mark.parametrize("dims,R,H", SHAPES)
def test_gradient_matches_oracle(dims, R, H, kernel):
    print("case: identity", dims, R, H, kernel, flush=True)
    prob = gi.random_dense(dims, R, H, "gaussian", seed=R + H, w=1.3, theta=0.8, lam=0.05, mu=0.2)
    G, gs = _grad(prob, kernel=kernel)
    Gr, gsr = og.gradient(prob.promoted())
    for k in range(3):
        assert grad_err(G[k], Gr[k]) <= TOL, k
    assert grad_err(gs, gsr) <= TOL


def test_fp64_and_model_history():
    print("case: identity fp64 / model history", flush=True)
    p64 = gi.random_dense((7, 9, 70), 6, 3, "gaussian", seed=2, lam=0.1, mu=0.1, dtype=np.float64)
    G, gs = _grad(p64)
    Gr, gsr = og.gradient(p64)
    assert max(grad_err(G[k], Gr[k]) for k in range(3)) <= 1e-12 and grad_err(gs, gsr) <= 1e-12
    pm = gi.random_dense((11, 6, 33), 4, 3, "gaussian", seed=5, lam=0.05, mu=0.1, dtype=np.float64)
    pm.A_old = [a + 0.1 for a in pm.A]
    import torch
    from paper_2110_14514_amd import Stream
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(pm.dims, 4, 3, "gaussian", [T(a) for a in pm.A_old], [], T(pm.s_hist), list(pm.t_hist),
                hist="model", lam=0.05, mu=0.1, gauss_identity=True)
    _, G, gs = st.loss_grad(T(pm.X_t), [T(a) for a in pm.A], T(pm.s_t), want_loss=False)
    assert st.sync() == 0
    Gr, gsr = omh.gradient_model(pm)
    assert max(grad_err(G[k].cpu().numpy(), Gr[k]) for k in range(3)) <= 1e-12
    assert grad_err(gs.cpu().numpy(), gsr) <= 1e-12


def test_objective_calls_are_unchanged():
    """Calls that ask for the objective take the model path: bitwise equal
    to a stream without the flag."""
    import torch
    print("case: identity objective", flush=True)
    prob = gi.random_dense((17, 33, 129), 16, 3, "gaussian", seed=4)
    dev = to_device(prob)
    a = make_stream(prob, dev, gauss_identity=True).loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    b = make_stream(prob, dev).loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and all(torch.equal(x, y) for x, y in zip(a[1], b[1]))


@pytest.mark.parametrize("kappa_f", [0, 3])
def test_stream_steps_match_oracle(kappa_f):
    """Three Gaussian OnlineGCP steps (LS weights, factor updates through the
    identity, with and without Algorithm 4's epochs) in FP64."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: identity steps", kappa_f, flush=True)
    prob = gi.random_dense((20, 30, 40), 4, 3, "gaussian", seed=8, dtype=np.float64)
    kw = dict(w=1.1, theta=0.9, lam=0.05, mu=0.1, tau_f=2, alpha_f=0.05, seed=3, kappa_f=kappa_f)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(prob.dims, 4, 3, "gaussian", [T(a) for a in prob.A], [T(x) for x in prob.X_hist],
                T(prob.s_hist), list(prob.t_hist), gauss_identity=True, **kw)
    orc = StreamOracle(prob.A, prob.X_hist, prob.s_hist, prob.t_hist, loss="gaussian", window=3, **kw)
    g = np.random.default_rng(12)
    for step in range(3):
        X = g.normal(size=prob.dims)
        s = st.step(T(X))
        s_ref = orc.step(X)
        assert st.sync() == 0
        assert rel_err(s.cpu().numpy(), s_ref) <= 1e-9
        for k, a in enumerate(st.factors()):
            assert rel_err(a.cpu().numpy(), orc.A[k]) <= 1e-9, (step, k)
