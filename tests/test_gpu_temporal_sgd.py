"""Device-side temporal-weight SGD (Algorithm 3 with the ADAM Step and the
epoch roll-back of Algorithm 2) against the FP64 oracle: iterates, objective,
roll-back decisions, rate and iteration count; stopping test, bound, batch
and graph capture."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import temporal_sgd as ots

from helpers import rel_err

pytestmark = pytest.mark.gpu

# several 64-wide mode-3 chunks with a ragged last one, one partial chunk,
# and exact chunks with row groups that do not divide the rows
SHAPES = [(9, 7, 150), (5, 3, 40), (33, 17, 128)]
# initial rate per loss: large enough that the first epoch raises the
# objective and is rolled back on these instances
ALPHA = {"gaussian": 10.0, "poisson_log": 10.0, "bernoulli_logit": 20.0}


def _stream(dims, R, loss, A, dtype, **kw):
    import torch
    from paper_2110_14514_amd import Stream
    dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype) for a in A]
    return Stream(dims, R, 0, loss, dev, tsolve="sgd", **kw)


def _solve(dims, R, loss, dtype, seed, *, mu=0.1, lower=-np.inf, alpha=1.0, tau=6, kappa=5, tol=-np.inf):
    import torch
    npdt = np.float64 if dtype == torch.float64 else np.float32
    X, A, _ = gi.weight_problem(dims, R, loss, seed, dtype=npdt)
    st = _stream(dims, R, loss, A, dtype, mu=mu, lower=lower, alpha_w=alpha, tau_w=tau, kappa_w=kappa,
                 tol_w=tol)
    Xd = torch.from_numpy(X).to("cuda")
    s = st.solve_st(Xd)
    info = st.solve_info()
    code = st.sync()
    ref, rinfo = ots.temporal_sgd(X.astype(np.float64), [a.astype(np.float64) for a in A], loss, mu=mu,
                                  lower=lower, alpha=alpha, tau=tau, kappa=kappa, tol=tol)
    return s.double().cpu().numpy(), info, code, ref, rinfo, (st, Xd)


def _clear_decisions(rinfo, margin):
    """The instance is usable for a comparison of decisions only if every
    epoch's objective differs from the accepted one by more than the
    rounding of either side."""
    F_old = rinfo.F[:-1]
    return all(abs(t - f) > margin * abs(f) for t, f in zip(rinfo.F_try, F_old))


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
@pytest.mark.parametrize("R", [5, 20, 40])
@pytest.mark.parametrize("dims", SHAPES)
def test_fp64_matches_oracle(dims, R, loss):
    import torch
    print("case: fp64", dims, R, loss, flush=True)
    s, info, code, ref, rinfo, _ = _solve(dims, R, loss, torch.float64, seed=R + len(dims) + dims[2], alpha=1.0)
    assert code == 0
    assert _clear_decisions(rinfo, 1e-10)
    assert info["rolled"] == rinfo.rolled
    assert info["epochs"] == len(rinfo.rolled)
    assert info["iters"] == rinfo.iters
    assert info["alpha"] == pytest.approx(rinfo.alpha, rel=1e-15)
    assert abs(info["F"] - rinfo.F[-1]) <= 1e-11 * abs(rinfo.F[-1])
    assert rel_err(s, ref) <= 1e-9


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
def test_fp64_first_epoch_rolled_back(loss):
    """A rate that overshoots: the first epoch raises F, is undone, and the
    solve continues with the rate divided by ten."""
    import torch
    print("case: rollback", loss, flush=True)
    s, info, code, ref, rinfo, _ = _solve((9, 7, 150), 5, loss, torch.float64, seed=11, alpha=ALPHA[loss])
    assert code == 0
    assert _clear_decisions(rinfo, 1e-10)
    assert rinfo.rolled[0] and info["rolled"] == rinfo.rolled
    assert info["alpha"] == pytest.approx(rinfo.alpha, rel=1e-15)
    assert info["iters"] == rinfo.iters
    assert rel_err(s, ref) <= 1e-9


@pytest.mark.parametrize("loss", ["gaussian", "poisson_log", "bernoulli_logit"])
@pytest.mark.parametrize("dims", SHAPES)
def test_fp32_matches_oracle(dims, loss):
    """FP32 solve far from stationarity: the same decisions, iterates within
    the FP32 tolerance carried through the ADAM steps."""
    import torch
    print("case: fp32", dims, loss, flush=True)
    s, info, code, ref, rinfo, _ = _solve(dims, 8, loss, torch.float32, seed=5 + dims[0], alpha=0.03, tau=6,
                                          kappa=3)
    assert code == 0
    assert _clear_decisions(rinfo, 1e-4)
    assert info["rolled"] == rinfo.rolled and info["iters"] == rinfo.iters
    assert abs(info["F"] - rinfo.F[-1]) <= 1e-5 * abs(rinfo.F[-1])
    assert rel_err(s, ref) <= 1e-4


def test_fp32_rollback_then_progress():
    import torch
    print("case: fp32 rollback", flush=True)
    s, info, code, ref, rinfo, _ = _solve((9, 7, 150), 5, "poisson_log", torch.float32, seed=11, alpha=10.0,
                                          tau=6, kappa=3)
    assert code == 0
    assert _clear_decisions(rinfo, 1e-4)
    assert rinfo.rolled[0] and info["rolled"] == rinfo.rolled
    assert rel_err(s, ref) <= 1e-4


def test_stopping_tolerance():
    """while F > tol_w: a tolerance above F(0) runs no epoch and returns
    s = 0; one between the epochs' objectives stops where the oracle does."""
    import torch
    print("case: tolerance", flush=True)
    dims, R, loss = (9, 7, 150), 5, "poisson_log"
    _, _, _, _, full, _ = _solve(dims, R, loss, torch.float64, seed=3, alpha=0.1)
    s, info, code, ref, rinfo, _ = _solve(dims, R, loss, torch.float64, seed=3, alpha=0.1, tol=full.F[0] + 1.0)
    assert code == 0 and info["epochs"] == 0 and not np.any(s) and info["F"] == pytest.approx(full.F[0])
    tol = 0.5 * (full.F[2] + full.F[3])
    s, info, code, ref, rinfo, _ = _solve(dims, R, loss, torch.float64, seed=3, alpha=0.1, tol=tol)
    assert len(rinfo.rolled) == 3 and info["epochs"] == 3
    assert rel_err(s, ref) <= 1e-9


def test_no_epochs():
    import torch
    print("case: kappa 0", flush=True)
    s, info, code, ref, rinfo, _ = _solve((5, 3, 40), 4, "bernoulli_logit", torch.float64, seed=2, kappa=0)
    assert code == 0 and info["epochs"] == 0 and info["iters"] == 0 and not np.any(s)
    assert info["F"] == pytest.approx(rinfo.F[0], rel=1e-12)


def test_lower_bound():
    """The ADAM Step clamps to the bound l (nonnegative weights)."""
    import torch
    print("case: lower", flush=True)
    s, info, code, ref, rinfo, _ = _solve((9, 7, 150), 6, "gaussian", torch.float64, seed=9, alpha=1.0,
                                          lower=1.5)
    assert code == 0 and np.all(s >= 1.5) and np.sum(s == 1.5) == np.sum(ref == 1.5) >= 1
    assert info["rolled"] == rinfo.rolled
    assert rel_err(s, ref) <= 1e-9


def test_repeatable_and_restartable():
    """Fixed-order sums: two solves give the same bits, and a solve starts
    from scratch whatever the previous one left."""
    import torch
    print("case: repeat", flush=True)
    s1, i1, _, _, _, (st, Xd) = _solve((33, 17, 128), 20, "poisson_log", torch.float32, seed=4, alpha=0.05)
    s2 = st.solve_st(Xd).double().cpu().numpy()
    assert np.array_equal(s1, s2) and st.solve_info() == i1


def test_full_step_matches_oracle_stream():
    """One OnlineGCP time step with the SGD temporal solve (Algorithm 1 with
    Algorithm 3) for a Poisson stream with a window: weights, then factors."""
    import torch
    from oracle.stream import StreamOracle
    from paper_2110_14514_amd import Stream
    print("case: full step", flush=True)
    prob = gi.random_dense((12, 10, 70), 6, 3, "poisson_log", seed=21, dtype=np.float64)
    kw = dict(alpha_f=1e-2, tau_f=2, mu=0.05, lam=0.02, w=1.2, theta=0.9, seed=5)
    sgd = dict(tsolve="sgd", tau_w=5, kappa_w=4, alpha_w=0.05)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    st = Stream(prob.dims, prob.rank, 3, "poisson_log", [T(a) for a in prob.A], [T(x) for x in prob.X_hist],
                T(prob.s_hist), [int(t) for t in prob.t_hist], **kw, **sgd)
    ref = StreamOracle(prob.A, prob.X_hist, prob.s_hist, prob.t_hist, loss="poisson_log", window=3, **kw, **sgd)
    s_ref = ref.solve_st(prob.X_t)
    ref.update_factors(prob.X_t, s_ref)
    s = st.step(T(prob.X_t))
    assert st.sync() == 0
    assert st.solve_info()["rolled"] == ref.solve_info.rolled
    assert rel_err(s.cpu().numpy(), s_ref) <= 1e-9
    for k, a in enumerate(st.factors()):
        assert rel_err(a.cpu().numpy(), ref.A[k]) <= 1e-9


def test_batch_solve_and_graph_replay():
    """Batched temporal solve: SGD streams get the per-stream result bitwise;
    a captured solve replayed with new slices copied in between equals the
    eager solves."""
    import torch
    from paper_2110_14514_amd import Batch
    print("case: batch sgd", flush=True)
    specs = [((23, 17, 70), 16, "poisson_log"), ((9, 9, 129), 8, "bernoulli_logit"),
             ((40, 33, 41), 12, "poisson_log")]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        streams, data = [], []
        for i, (dims, R, loss) in enumerate(specs):
            X, A, _ = gi.weight_problem(dims, R, loss, 30 + i)
            streams.append(_stream(dims, R, loss, A, torch.float32, mu=0.1, alpha_w=0.05, tau_w=4, kappa_w=3))
            X2, _, _ = gi.weight_problem(dims, R, loss, 40 + i)
            data.append((torch.from_numpy(X).cuda(), torch.from_numpy(X2).cuda()))
        Xb = [d[0].clone() for d in data]
        Sb = [torch.zeros(st.rank, device="cuda") for st in streams]
    torch.cuda.synchronize()
    b = Batch(streams, Xb, Sb)
    with torch.cuda.stream(side):
        b.solve_st()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    for i, st in enumerate(streams):
        with torch.cuda.stream(side):
            ref = st.solve_st(data[i][0])
        torch.cuda.synchronize()
        assert torch.equal(Sb[i], ref), i
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=side):
        b.solve_st()
    for rep in range(3):
        with torch.cuda.stream(side):
            for i in range(len(specs)):
                Xb[i].copy_(data[i][rep % 2])
            cg.replay()
        torch.cuda.synchronize()
        for i, st in enumerate(streams):
            with torch.cuda.stream(side):
                ref = st.solve_st(data[i][rep % 2])
            torch.cuda.synchronize()
            assert torch.equal(Sb[i], ref), (rep, i)
    assert b.sync_streams() == 0


def test_c2_size_weight_solve():
    """The C2 shape (200 x 200 x 200 Poisson-count slice, rank 16) in the
    bench's launch configuration, with a short solve the FP64 oracle finishes
    in seconds: decisions, objective and weights."""
    import torch
    print("case: c2 weight solve", flush=True)
    dims, R = (200, 200, 200), 16
    X, A, _ = gi.weight_problem(dims, R, "poisson_log", 1)
    st = _stream(dims, R, "poisson_log", A, torch.float32, tau_w=3, kappa_w=2, alpha_w=0.05)
    s = st.solve_st(torch.from_numpy(X).cuda()).double().cpu().numpy()
    info = st.solve_info()
    assert st.sync() == 0
    ref, rinfo = ots.temporal_sgd(X.astype(np.float64), [a.astype(np.float64) for a in A], "poisson_log",
                                  alpha=0.05, tau=3, kappa=2)
    assert _clear_decisions(rinfo, 1e-4)
    assert info["rolled"] == rinfo.rolled
    assert abs(info["F"] - rinfo.F[-1]) <= 1e-5 * abs(rinfo.F[-1])
    assert rel_err(s, ref) <= 1e-4
