"""gcp_loss_grad_static (the entry point for callers that cannot allocate:
partial sums in the library's fixed per-GPU array) against gcp_loss_grad on
the same inputs, on two calls in a row, the second with a smaller input, and
against the oracle."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og

from helpers import TOL, compare, make_stream, to_device

pytestmark = pytest.mark.gpu


def _static(prob, dev, out, kernel="auto"):
    import torch
    from paper_2110_14514_amd.stream import loss_grad_static
    H = len(prob.X_hist)
    Xh = torch.stack(dev["X_hist"]).contiguous() if H else None
    return loss_grad_static(prob.dims, prob.rank, prob.loss, dev["X_t"], dev["A"], dev["s_t"], Xh, dev["s_hist"],
                            list(prob.t_hist), prob.t, w=prob.w, theta=prob.theta, lam=prob.lam, mu=prob.mu,
                            kernel=kernel, out=out)


@pytest.mark.parametrize("kernel", ["mfma", "valu"])
def test_static_entry_matches_loss_grad_on_two_calls(kernel):
    import torch
    print("case: static entry", kernel, flush=True)
    probs = [gi.random_dense((37, 45, 70), 16, 3, "poisson_log", seed=61, w=1.2, theta=0.9, lam=0.05, mu=0.1),
             gi.random_dense((9, 10, 33), 8, 2, "gaussian", seed=62, w=0.8, theta=0.95, lam=0.1, mu=0.2)]
    R = max(p.rank for p in probs)
    dmax = [max(p.dims[k] for p in probs) for k in range(3)]
    # output buffers made once, before the calls: the calls themselves allocate nothing
    big = (torch.empty(1, device="cuda"), [torch.empty(dmax[k] * R, device="cuda") for k in range(3)],
           torch.empty(R, device="cuda"))
    for prob in probs:
        dev = to_device(prob)
        st = make_stream(prob, dev, kernel=kernel)
        loss_r, G_r, gs_r = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
        out = (big[0], [big[1][k][: prob.dims[k] * prob.rank].view(prob.dims[k], prob.rank) for k in range(3)],
               big[2][: prob.rank])
        loss_s, G_s, gs_s = _static(prob, dev, out, kernel)
        torch.cuda.synchronize()
        assert st.sync() == 0
        ref = (float(loss_r.item()), [g.double().cpu().numpy() for g in G_r], gs_r.double().cpu().numpy())
        got = (float(loss_s.item()), [g.double().cpu().numpy() for g in G_s], gs_s.double().cpu().numpy())
        # against the existing entry point (same kernels and summation order)
        assert abs(got[0] - ref[0]) <= TOL * max(abs(ref[0]), 1.0)
        for k in range(3):
            np.testing.assert_allclose(got[1][k], ref[1][k], rtol=0, atol=TOL * np.max(np.abs(ref[1][k])))
        np.testing.assert_allclose(got[2], ref[2], rtol=0, atol=TOL * np.max(np.abs(ref[2])))
        # and against the oracle
        errs = compare(prob, got, og)
        assert max(errs.values()) <= TOL, errs


def test_static_entry_fp64_and_gradient_only():
    import torch
    print("case: static entry fp64 / gradient only", flush=True)
    prob = gi.random_dense((11, 13, 52), 12, 4, "bernoulli_logit", seed=63, lam=0.05, mu=0.1, dtype=np.float64)
    dev = to_device(prob)
    loss, G, gs = _static(prob, dev, None)
    torch.cuda.synchronize()
    errs = compare(prob, (float(loss.item()), [g.cpu().numpy() for g in G], gs.cpu().numpy()), og)
    assert max(errs.values()) <= 1e-12, errs
    from paper_2110_14514_amd.stream import loss_grad_static
    Xh = torch.stack(dev["X_hist"]).contiguous()
    _, G2, gs2 = loss_grad_static(prob.dims, prob.rank, prob.loss, dev["X_t"], dev["A"], dev["s_t"], Xh,
                                  dev["s_hist"], list(prob.t_hist), prob.t, lam=prob.lam, mu=prob.mu,
                                  want_loss=False)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(G2[k], G[k])
    assert torch.equal(gs2, gs)
