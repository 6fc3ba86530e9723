"""GPU parity of the stratified sampled path (COO slices) against the FP64
oracle, which regenerates the same Philox draws independently."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import sampled as osm
from oracle.adam import adam_step

from helpers import TOL, loss_err, grad_err, rel_err

pytestmark = pytest.mark.gpu


def _dev_coo(sl):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(sl.coords, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sl.vals, dtype=np.float32)).cuda())


def _stream(prob, **kw):
    import torch
    from paper_2110_14514_amd import Stream
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    hist = [_dev_coo(x) for x in prob.X_hist]
    max_nnz = max([x.coords.shape[0] for x in [prob.X_t] + list(prob.X_hist)])
    st = Stream(prob.dims, prob.rank, len(prob.X_hist), prob.loss, [T(a) for a in prob.A], hist,
                T(prob.s_hist) if len(hist) else None, list(prob.t_hist), w=prob.w,
                theta=prob.theta, lam=prob.lam, mu=prob.mu, seed=prob.seed, slice_kind="coo",
                max_nnz=max_nnz, p=prob.p, q=prob.q, **kw)
    return st, T


def _f32(prob):
    """The oracle sees the FP32 inputs promoted exactly."""
    prob.A = [a.astype(np.float32).astype(np.float64) for a in prob.A]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    prob.s_hist = prob.s_hist.astype(np.float32).astype(np.float64)
    for sl in [prob.X_t] + list(prob.X_hist):
        sl.vals = sl.vals.astype(np.float32).astype(np.float64)
    return prob


CASES = [
    ((30, 40, 50), 8, 3, 2000, 3000, 3000, "poisson_log"),
    ((30, 40, 50), 16, 2, 1500, 2500, 4000, "bernoulli_logit"),
    ((21, 33, 17), 32, 4, 900, 1000, 2000, "gaussian"),
    ((13, 9, 70), 48, 1, 400, 777, 333, "poisson_log"),
    ((40, 40, 40), 12, 0, 5000, 0, 4096, "poisson_log"),   # zeros only
    ((40, 40, 40), 12, 2, 5000, 4096, 0, "poisson_log"),   # nonzeros only
    # the paper's count-data shapes: 263 x 263 x 24 at 3.8% density, rank 50,
    # window 30, 10k + 10k draws; 24 x 77 x 32 at 1.6%, rank 50, as many
    # nonzero draws as nonzeros plus 1k zeros, window at the library's maximum
    ((263, 263, 24), 50, 30, 63000, 10000, 10000, "poisson_log"),
    ((24, 77, 32), 50, 64, 946, 946, 1000, "poisson_log"),
]


@pytest.mark.parametrize("reduction", ["sorted", "atomic"])
@pytest.mark.parametrize("dims,R,H,nnz,p,q,loss", CASES)
def test_sampled_matches_oracle(dims, R, H, nnz, p, q, loss, reduction):
    """Both ways of summing the MTTKRP rows (row-sorted lists, float atomics)."""
    import torch
    print("case: sampled", reduction, dims, R, H, nnz, p, q, loss, flush=True)
    prob = _f32(gi.sparse_problem(dims=dims, rank=R, window=H, nnz=nnz, p=p, q=q, seed=R + H,
                                  loss=loss))
    prob.lam, prob.mu, prob.theta, prob.w = 0.05, 0.1, 0.9, 1.3
    st, T = _stream(prob, sampled_atomic=reduction == "atomic")
    Xt = _dev_coo(prob.X_t)
    A = [T(a) for a in prob.A]
    for call in range(2):
        loss_v, G, g_s = st.loss_grad(Xt, A, T(prob.s_t))
        torch.cuda.synchronize()
        assert st.sync() == 0
        assert st.info()["sample_call"] == call + 1
        F, Gr, gsr = osm.sampled_loss_grad(prob, call=call)
        scale = max(abs(F), 1.0)
        assert loss_err(loss_v.item(), F, scale) <= TOL
        for k in range(3):
            assert grad_err(G[k].double().cpu().numpy(), Gr[k]) <= TOL, (call, k)
        assert grad_err(g_s.double().cpu().numpy(), gsr) <= TOL


def test_sampled_update_factors_matches_oracle():
    """Two Adam iterations on sampled gradients (calls 0 and 1), then the
    window push of the COO slice."""
    import torch
    print("case: sampled update", flush=True)
    prob = _f32(gi.sparse_problem(dims=(25, 30, 35), rank=8, window=2, nnz=1200, p=1500, q=1500,
                                  seed=5, loss="poisson_log"))
    st, T = _stream(prob, alpha_f=1e-2, tau_f=2)
    st.update_factors(_dev_coo(prob.X_t), T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    A = [a.copy() for a in prob.A]
    u = [np.zeros_like(a) for a in A]
    v = [np.zeros_like(a) for a in A]
    for it in range(2):
        prob.A = A
        _, G, _ = osm.sampled_loss_grad(prob, call=it)
        for k in range(3):
            A[k], u[k], v[k] = adam_step(A[k], G[k], u[k], v[k], it, 1e-2)
    got = [a.double().cpu().numpy() for a in st.factors()]
    for k in range(3):
        assert rel_err(got[k], A[k]) <= 1e-5
    info = st.info()
    assert info["t"] == prob.t + 1 and info["sample_call"] == 2
    assert info["n_window"] == 2          # window already full: reservoir kept or replaced


def test_dump_samples_equal_the_oracle_draws():
    """gcp_dump_samples returns the draws the gradient kernels form (the same
    device code): they equal the oracle's draws from the published
    generator, for the current slice and the window slots, at two call
    numbers, and the stream's call counter does not move."""
    print("case: sample dump", flush=True)
    prob = _f32(gi.sparse_problem(dims=(30, 40, 50), rank=8, window=2, nnz=2000, p=3000, q=3000, seed=3,
                                  loss="poisson_log"))
    st, T = _stream(prob)
    Xt = _dev_coo(prob.X_t)
    for h in range(3):
        sl = prob.X_t if h == 0 else prob.X_hist[h - 1]
        stamp = prob.t if h == 0 else int(prob.t_hist[h - 1])
        for call in (0, 5):
            coords, w = st.dump_samples(Xt, h, call)
            c_or, _, w_or = osm.sampled_terms(prob.loss, sl, None, None, prob.seed, stamp, call, prob.p, prob.q)
            assert np.array_equal(coords.cpu().numpy(), c_or.astype(np.int32)), (h, call)
            assert np.allclose(w.cpu().numpy(), w_or, rtol=1e-6), (h, call)
            # zero draws avoid the stored entries; nonzero draws are stored entries
            d = prob.dims
            lin = lambda c: (c[:, 0].astype(np.int64) * d[1] + c[:, 1]) * d[2] + c[:, 2]
            stored = set(lin(sl.coords).tolist())
            got = lin(coords.cpu().numpy())
            assert all(v in stored for v in got[:prob.p].tolist())
            assert not any(v in stored for v in got[prob.p:].tolist())
    assert st.sync() == 0
    assert st.info()["sample_call"] == 0


def test_dump_samples_are_uniform():
    """Chi-square checks of the sampler on the device: nonzero draws uniform
    over the stored entries, zero draws uniform over the other cells (fixed
    seeds; thresholds at the 0.1% tail of the chi-square law)."""
    from scipy.stats import chi2
    print("case: sample uniformity", flush=True)
    prob = _f32(gi.sparse_problem(dims=(4, 5, 6), rank=4, window=0, nnz=20, p=100_000, q=100_000, seed=9,
                                  loss="poisson_log"))
    st, T = _stream(prob)
    coords, _ = st.dump_samples(_dev_coo(prob.X_t), 0, 0)
    c = coords.cpu().numpy().astype(np.int64)
    lin = (c[:, 0] * 5 + c[:, 1]) * 6 + c[:, 2]
    stored = (prob.X_t.coords[:, 0].astype(np.int64) * 5 + prob.X_t.coords[:, 1]) * 6 + prob.X_t.coords[:, 2]
    counts = np.bincount(lin, minlength=120)
    nz = counts[stored]
    zmask = np.ones(120, bool)
    zmask[stored] = False
    zc = counts[zmask]
    assert nz.sum() >= prob.p and zc.sum() == prob.q
    for obs in (np.bincount(np.searchsorted(np.sort(stored), lin[:prob.p]), minlength=len(stored)), zc):
        exp = obs.sum() / len(obs)
        stat = float(np.sum((obs - exp) ** 2 / exp))
        assert stat < chi2.ppf(0.999, len(obs) - 1), stat


@pytest.mark.parametrize("alpha,expect_roll", [(1e-2, False), (1.0, True), (0.3, False)])
def test_sampled_factor_epochs_match_oracle(alpha, expect_roll):
    """Algorithm 4 on COO slices: sampled gradients (new draws each step),
    epochs judged by Algorithm 5's estimate over draws fixed for the solve,
    decisions and factors equal to the oracle's."""
    import torch
    from types import SimpleNamespace
    print("case: sampled epochs", alpha, flush=True)
    prob = _f32(gi.sparse_problem(dims=(25, 30, 35), rank=8, window=2, nnz=1200, p=1500, q=1500,
                                  seed=5, loss="poisson_log"))
    st, T = _stream(prob, alpha_f=alpha, tau_f=2, kappa_f=3, p_est=2000, q_est=2000)
    st.update_factors(_dev_coo(prob.X_t), T(prob.s_t))
    info = st.factor_info()
    assert st.sync() == 0
    A = [np.asarray(a, np.float64).copy() for a in prob.A]
    z = [np.zeros_like(a) for a in A]
    state = SimpleNamespace(A=A, u=[a.copy() for a in z], v=[a.copy() for a in z], Ao=[a.copy() for a in A],
                            uo=[a.copy() for a in z], vo=[a.copy() for a in z], alpha=alpha, i=0, call=0)
    rolled = osm.sampled_factor_epochs(prob, state, tau=2, kappa=3, p_est=2000, q_est=2000)
    assert rolled[0] == expect_roll
    # decisions far from ties compared with FP32 rounding of the estimates
    assert all(abs(t - f) > 1e-4 * abs(f) for t, f in zip(state.F_try, state.F_hist[:-1]))
    assert info["rolled"] == rolled and info["iters"] == state.i
    assert info["alpha"] == pytest.approx(state.alpha, rel=1e-15)
    assert abs(info["F"] - state.F) <= 1e-5 * abs(state.F)
    got = [a.double().cpu().numpy() for a in st.factors()]
    for k in range(3):
        assert rel_err(got[k], state.A[k]) <= 1e-5
    assert st.info()["sample_call"] == 6


@pytest.mark.parametrize("alpha", [0.05, 1.0])
def test_sampled_weight_solve_matches_oracle(alpha):
    """Algorithm 3 on a COO slice: sampled weight gradients of X_t alone,
    epochs judged by Algorithm 5's estimate; decisions, rate, index and
    weights equal the oracle's, and the call counter moves by tau kappa."""
    import torch
    print("case: sampled weight solve", alpha, flush=True)
    prob = _f32(gi.sparse_problem(dims=(25, 30, 35), rank=8, window=2, nnz=1200, p=1500, q=1500,
                                  seed=5, loss="poisson_log"))
    st, T = _stream(prob, tsolve="sgd", tau_w=3, kappa_w=3, alpha_w=alpha, p_est=2000, q_est=2000)
    s = st.solve_st(_dev_coo(prob.X_t))
    info = st.solve_info()
    assert st.sync() == 0
    ref, rinfo = osm.sampled_temporal_sgd(prob, 0, alpha=alpha, tau=3, kappa=3, p_est=2000, q_est=2000)
    assert all(abs(t - f) > 1e-4 * abs(f) for t, f in zip(rinfo.F_try, rinfo.F[:-1]))
    assert info["rolled"] == rinfo.rolled and info["iters"] == rinfo.iters
    assert info["alpha"] == pytest.approx(rinfo.alpha, rel=1e-15)
    assert abs(info["F"] - rinfo.F[-1]) <= 1e-5 * abs(rinfo.F[-1])
    assert rel_err(s.double().cpu().numpy(), ref) <= 1e-4
    assert st.info()["sample_call"] == 9


@pytest.mark.gpu
def test_sampled_larger_draw_counts_match_oracle():
    """263 x 263 x 24 at 3.8% density, rank 50, window 30 with 50k + 50k
    draws per slice (one call: the oracle takes about ten seconds).  With
    this many draws a wave of the draw kernel takes 4 x 64 of them and the
    reduction walks runs of 256 records; the smaller cases above take the
    short forms (64 draws per wave, shorter runs)."""
    print("case: sampled 263x263x24 R50 H30 p=q=50000", flush=True)
    prob = _f32(gi.sparse_problem(dims=(263, 263, 24), rank=50, window=30, nnz=63000, p=50000,
                                  q=50000, seed=80, loss="poisson_log"))
    st, T = _stream(prob)
    loss_v, G, g_s = st.loss_grad(_dev_coo(prob.X_t), [T(a) for a in prob.A], T(prob.s_t))
    assert st.sync() == 0
    F, Gr, gsr = osm.sampled_loss_grad(prob, call=0)
    assert loss_err(loss_v.item(), F, max(abs(F), 1.0)) <= TOL
    for k in range(3):
        assert grad_err(G[k].double().cpu().numpy(), Gr[k]) <= TOL, k
    assert grad_err(g_s.double().cpu().numpy(), gsr) <= TOL
