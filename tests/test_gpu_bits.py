"""Bit-packed binary slices (GCP_SLICE_BITS) on the GPU: objective and
gradients against the oracle on the same 0/1 data, against the FP32 slice
path of the same kernels (bit for bit: only the storage differs), and whole
time steps (window pushes of packed slices, the weights' SGD solve,
factor epochs) against the FP32 stream."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og

from helpers import TOL, compare, make_stream, rel_err, to_device

pytestmark = pytest.mark.gpu

# one and two h-tiles (window up to 31), I3 tails (16-entry half group,
# 33 and 70 entries), the single-slice kernel (window 0), ranks 4..32
CASES = [((23, 17, 70), 16, 4, "bernoulli_logit"), ((9, 9, 129), 32, 20, "bernoulli_logit"),
         ((31, 9, 33), 8, 7, "bernoulli_odds"), ((12, 40, 64), 32, 16, "bernoulli_logit"),
         ((5, 6, 7), 4, 0, "bernoulli_logit"), ((40, 33, 41), 12, 0, "bernoulli_odds"),
         ((17, 3, 45), 20, 31, "bernoulli_logit"), ((30, 20, 16), 16, 3, "bernoulli_logit"),
         ((30, 41, 200), 32, 0, "bernoulli_logit")]


def _problem(dims, R, H, loss, seed):
    if loss == "bernoulli_odds":
        return gi.nonneg_dense(dims, R, H, loss, seed=seed, w=1.1, theta=0.9, lam=0.05, mu=0.1)
    return gi.random_dense(dims, R, H, loss, seed=seed, w=1.1, theta=0.9, lam=0.05, mu=0.1)


def _bits(x):
    import torch
    return torch.from_numpy(gi.pack_bits(x).view(np.int32)).cuda()


def _bits_stream(p, dev, **kw):
    from paper_2110_14514_amd import Stream
    return Stream(p.dims, p.rank, len(p.X_hist), p.loss, dev["A"], [_bits(x) for x in p.X_hist],
                  dev["s_hist"], dev["t_hist"], w=p.w, theta=p.theta, lam=p.lam, mu=p.mu, slice_kind="bits", **kw)


@pytest.mark.parametrize("dims,R,H,loss", CASES)
def test_bits_loss_grad_matches_oracle_and_fp32_slices(dims, R, H, loss):
    import torch
    print("case: bits loss_grad", dims, R, H, loss, flush=True)
    p = _problem(dims, R, H, loss, seed=R + H)
    assert set(np.unique(p.X_t)) <= {0.0, 1.0}
    dev = to_device(p)
    sb = _bits_stream(p, dev)
    lb, Gb, gb = sb.loss_grad(_bits(p.X_t), dev["A"], dev["s_t"])
    sf = make_stream(p, dev, kernel="mfma")
    lf, Gf, gf = sf.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
    assert sb.sync() == 0 and sf.sync() == 0
    # same tiles and summation order; only the slices' storage differs
    assert np.array_equal(lb.cpu().numpy(), lf.cpu().numpy())
    for k in range(3):
        assert np.array_equal(Gb[k].cpu().numpy(), Gf[k].cpu().numpy()), k
    assert np.array_equal(gb.cpu().numpy(), gf.cpu().numpy())
    got = (float(lb.item()), [g.double().cpu().numpy() for g in Gb], gb.double().cpu().numpy())
    errs = compare(p, got, og)
    assert max(errs.values()) <= TOL, errs


def test_bits_window_memory_is_one_32nd():
    """A window of packed slices: the workspace shrinks by 31/32 of the FP32
    window (less one FP32 slice for the solvers that read values)."""
    from paper_2110_14514_amd import Stream
    from paper_2110_14514_amd.stream import gcp_workspace_size, make_params
    import torch
    dims, R, H = (200, 100, 64), 32, 20
    pb = make_params(dims, R, H, "bernoulli_logit", dtype=torch.float32, slice_kind="bits")
    pd = make_params(dims, R, H, "bernoulli_logit", dtype=torch.float32)
    nb, nd = gcp_workspace_size(pb), gcp_workspace_size(pd)
    omega = 200 * 100 * 64
    assert nd - nb >= H * omega * 4 - H * omega // 8 - omega * 4 - (1 << 20)


@pytest.mark.parametrize("tsolve", ["sgd", "ls"])
def test_bits_steps_match_fp32_stream(tsolve):
    """Three time steps (weights' solve, factor epochs, window push of the
    packed slice) agree with the FP32-slice stream."""
    import torch
    print("case: bits steps", tsolve, flush=True)
    p = _problem((24, 19, 45), 8, 3, "bernoulli_logit", seed=5)
    dev = to_device(p)
    kw = dict(alpha_f=1e-2, tau_f=2, kappa_f=2, seed=3)
    if tsolve == "sgd":
        kw.update(tsolve="sgd", tau_w=3, kappa_w=2, alpha_w=0.05)
    sb = _bits_stream(p, dev, kernel="mfma", **kw)
    sf = make_stream(p, dev, kernel="mfma", **kw)
    g = np.random.default_rng(9)
    for step in range(3):
        X = (g.random(p.dims) < 0.3).astype(np.float32)
        Xf = torch.from_numpy(X).cuda()
        s0 = torch.from_numpy(g.uniform(0.5, 1.5, p.rank).astype(np.float32)).cuda()
        sbv, sfv = s0.clone(), s0.clone()
        if tsolve == "sgd":
            sb.solve_st(_bits(X), sbv)
            sf.solve_st(Xf, sfv)
        sb.update_factors(_bits(X), sbv)
        sf.update_factors(Xf, sfv)
        torch.cuda.synchronize()
        assert sb.sync() == 0 and sf.sync() == 0
        assert np.array_equal(sbv.cpu().numpy(), sfv.cpu().numpy()), step
        assert sb.info()["slot_times"] == sf.info()["slot_times"]
        assert sb.factor_info() == sf.factor_info(), step
        for a, b in zip(sb.factors(), sf.factors()):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), step


def test_bits_slice_loss_and_local_loss():
    import torch
    print("case: bits metrics", flush=True)
    p = _problem((20, 30, 70), 8, 2, "bernoulli_logit", seed=4)
    dev = to_device(p)
    sb = _bits_stream(p, dev)
    sf = make_stream(p, dev)
    fb, qb = sb.slice_loss(_bits(p.X_t), dev["s_t"])
    ff, qf = sf.slice_loss(dev["X_t"], dev["s_t"])
    assert qb == qf == float(np.sum(p.X_t))
    assert fb == pytest.approx(ff, rel=1e-6)
    assert sb.local_loss(_bits(p.X_t), dev["s_t"]) == pytest.approx(sf.local_loss(dev["X_t"], dev["s_t"]), rel=1e-6)


def test_bits_rejects_fp32_slices():
    import torch
    p = _problem((8, 8, 40), 4, 1, "bernoulli_logit", seed=1)
    dev = to_device(p)
    sb = _bits_stream(p, dev)
    with pytest.raises(RuntimeError):
        sb.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
