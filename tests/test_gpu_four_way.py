"""Four-way slices (d = 4, I1 x I2 x I3 x I4): objective and gradients of
all four factors against the oracle's four-way evaluation; whole time steps
(least-squares weights, factor epochs, window pushes) against the oracle's
stream; slice loss and K-tensor score against the oracle's metrics."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import metrics as om
from oracle.stream import StreamOracle

from helpers import TOL, grad_err, loss_err, rel_err, to_device

pytestmark = pytest.mark.gpu

CASES = [((12, 9, 5, 7), 8, 3, "gaussian", "auto", "float32"),
         ((20, 16, 4, 16), 16, 5, "poisson_log", "mfma", "float32"),
         ((7, 8, 3, 11), 32, 2, "bernoulli_logit", "valu", "float32"),
         ((10, 10, 6, 6), 12, 0, "poisson_log", "auto", "float32"),
         ((33, 17, 2, 9), 20, 18, "gaussian", "mfma", "float32"),
         ((6, 7, 4, 5), 5, 2, "gaussian", "auto", "float64"),
         ((5, 6, 3, 4), 6, 2, "bernoulli_logit", "auto", "float64")]


def _stream(p, dev, **kw):
    from paper_2110_14514_amd import Stream
    return Stream(p.dims, p.rank, len(p.X_hist), p.loss, dev["A"], dev["X_hist"], dev["s_hist"], dev["t_hist"],
                  w=p.w, theta=p.theta, lam=p.lam, mu=p.mu, **kw)


@pytest.mark.parametrize("dims,R,H,loss,kernel,dtype", CASES)
def test_four_way_loss_grad_matches_oracle(dims, R, H, loss, kernel, dtype):
    import torch
    print("case: d4 loss_grad", dims, R, H, loss, kernel, dtype, flush=True)
    p = gi.random_dense(dims, R, H, loss, seed=R + H, w=1.1, theta=0.9, lam=0.05, mu=0.1,
                        dtype=np.float64 if dtype == "float64" else np.float32)
    dev = to_device(p)
    st = _stream(p, dev, kernel=kernel)
    lv, G, gs = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
    assert st.sync() == 0 and len(G) == 4
    p64 = p.promoted()
    F = og.objective(p64)
    Gr, gsr = og.gradient(p64)
    tol = TOL if dtype == "float32" else 1e-12
    assert loss_err(lv.item(), F, og.loss_terms_abs(p64)) <= tol
    for k in range(4):
        assert G[k].shape == (dims[k], R)
        assert grad_err(G[k].double().cpu().numpy(), Gr[k]) <= tol, k
    assert grad_err(gs.double().cpu().numpy(), gsr) <= tol
    # loss only and gradient only give the same numbers
    lv2, _, _ = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], want_grad=False)
    _, G2, gs2 = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], want_loss=False)
    torch.cuda.synchronize()
    assert lv2.item() == lv.item()
    for k in range(4):
        assert np.array_equal(G2[k].cpu().numpy(), G[k].cpu().numpy())


@pytest.mark.parametrize("loss,kw", [("gaussian", dict(kappa_f=2, tau_f=2)),
                                     ("poisson_log", dict(tau_f=3, tsolve="sgd", tau_w=4, kappa_w=2,
                                                          alpha_w=0.05))])
def test_four_way_steps_match_oracle_stream(loss, kw):
    """Three OnlineGCP steps on four-way slices in FP64: weights (least
    squares or Algorithm 3), factor iterations or epochs, window pushes."""
    import torch
    print("case: d4 steps", loss, flush=True)
    dims, R, H = (9, 8, 4, 5), 4, 2
    p = gi.random_dense(dims, R, H, loss, seed=3, w=1.1, theta=0.9, lam=0.05, mu=0.1, dtype=np.float64)
    dev = to_device(p)
    common = dict(alpha_f=0.02, seed=5, **kw)
    st = _stream(p, dev, **common)
    orc = StreamOracle(p.A, p.X_hist, p.s_hist, list(p.t_hist), loss=loss, window=H, w=p.w, theta=p.theta,
                       lam=p.lam, mu=p.mu, d=4, **common)
    g = np.random.default_rng(11)
    for step in range(3):
        X = (g.normal(size=dims) if loss == "gaussian" else g.poisson(1.0, size=dims).astype(float))
        Xd = torch.from_numpy(X).cuda()
        sv = st.step(Xd)
        sr = orc.step(X)
        assert st.sync() == 0
        assert rel_err(sv.cpu().numpy(), sr) <= 1e-9, step
        F = st.factors()
        assert len(F) == 4
        for k in range(4):
            assert rel_err(F[k].cpu().numpy(), orc.A[k]) <= 1e-9, (step, k)
        assert st.info()["slot_times"] == list(orc.slots)


def test_four_way_metrics_match_oracle():
    import torch
    print("case: d4 metrics", flush=True)
    p = gi.random_dense((8, 9, 3, 7), 5, 1, "gaussian", seed=4, dtype=np.float64)
    dev = to_device(p)
    st = _stream(p, dev)
    f, q = st.slice_loss(dev["X_t"], dev["s_t"])
    fr, qr = om.slice_loss(p.X_t, p.A, p.s_t, "gaussian")
    assert f == pytest.approx(fr, rel=1e-12) and q == pytest.approx(qr, rel=1e-12)
    g = np.random.default_rng(2)
    B = [g.normal(size=(n, 4)) for n in (8, 9, 3, 7)]
    wb = g.uniform(0.5, 2.0, 4)
    score = st.ktensor_score(dev["s_t"], [torch.from_numpy(b).cuda() for b in B], torch.from_numpy(wb).cuda())
    assert score == pytest.approx(om.ktensor_score(p.A, p.s_t, B, wb), rel=1e-10)
