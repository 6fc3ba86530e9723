"""Batched multi-stream path: one persistent launch over streams of uneven
shapes, ranks, windows and losses; device-resident time steps; HIP-graph
capture and replay."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og

from helpers import TOL, compare, make_stream, rel_err, to_device

pytestmark = pytest.mark.gpu

# uneven shapes (ragged tiles, I3 tails, odd I3), ranks 8/12/16/32, windows
# 0..20 (one and two h-tiles), Gaussian / Poisson / Bernoulli
SPECS = [((23, 17, 70), 16, 4, "gaussian"), ((31, 9, 33), 8, 7, "poisson_log"),
         ((12, 40, 64), 32, 16, "poisson_log"), ((50, 6, 5), 12, 0, "gaussian"),
         ((9, 9, 129), 32, 20, "bernoulli_logit"), ((40, 33, 41), 16, 3, "poisson_log")]


def _problems():
    return [gi.random_dense(d, R, H, loss, seed=10 + i, w=1.1, theta=0.9, lam=0.05, mu=0.1)
            for i, (d, R, H, loss) in enumerate(SPECS)]


def _make(probs, **kw):
    devs = [to_device(p) for p in probs]
    streams = [make_stream(p, d, kernel="mfma", **kw) for p, d in zip(probs, devs)]
    return devs, streams


def test_batch_loss_grad_matches_streams_and_oracle():
    import torch
    from paper_2110_14514_amd import Batch
    print("case: batch loss_grad", flush=True)
    probs = _problems()
    devs, streams = _make(probs)
    Xb = [d["X_t"].clone() for d in devs]
    Sb = [d["s_t"].clone() for d in devs]
    b = Batch(streams, Xb, Sb)
    outs = b.loss_grad()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    for i, (p, d, st) in enumerate(zip(probs, devs, streams)):
        loss, G, g_s = st.loss_grad(d["X_t"], d["A"], d["s_t"])
        torch.cuda.synchronize()
        bl, bG, bg = outs[i]
        # same tile code and summation order; the history weights w theta^(t-h)
        # come from the device's pow here and the host's in the per-stream call
        assert rel_err(bl.cpu().numpy(), loss.cpu().numpy()) <= 1e-6, i
        for k in range(3):
            assert rel_err(bG[k].cpu().numpy(), G[k].cpu().numpy()) <= 1e-6, (i, k)
        assert rel_err(bg.cpu().numpy(), g_s.cpu().numpy()) <= 1e-6, i
        got = (float(bl.item()), [g.double().cpu().numpy() for g in bG], bg.double().cpu().numpy())
        errs = compare(p, got, og)
        assert max(errs.values()) <= TOL, (i, errs)


def _run_steps(use_batch, graph, nsteps=4, kappa_f=0):
    """nsteps OnlineGCP factor updates with fresh X_t/s_t each step
    (kappa_f > 0: Algorithm 4's epochs with the device-side decisions)."""
    import torch
    from paper_2110_14514_amd import Batch
    probs = _problems()
    side = torch.cuda.Stream()       # graph capture needs a non-default stream
    with torch.cuda.stream(side):
        devs, streams = _make(probs, alpha_f=1e-2, tau_f=2, seed=7, kappa_f=kappa_f)
    torch.cuda.synchronize()
    g = np.random.default_rng(3)
    data = [[(g.normal(size=p.dims).astype(np.float32) if p.loss == "gaussian" else
              g.poisson(1.0, size=p.dims).astype(np.float32) if p.loss == "poisson_log" else
              (g.random(p.dims) < 0.3).astype(np.float32),
              g.uniform(0.5, 1.5, size=p.rank).astype(np.float32)) for p in probs]
            for _ in range(nsteps)]
    Xb = [d["X_t"].clone() for d in devs]
    Sb = [d["s_t"].clone() for d in devs]
    cs = streams[0].hip_stream
    if use_batch:
        b = Batch(streams, Xb, Sb)
        cg = None
        for t in range(nsteps):
            with torch.cuda.stream(cs):
                for i in range(len(probs)):
                    Xb[i].copy_(torch.from_numpy(data[t][i][0]))
                    Sb[i].copy_(torch.from_numpy(data[t][i][1]))
            if graph:
                if cg is None:
                    torch.cuda.synchronize()
                    cg = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(cg, stream=cs):
                        b.update_factors()
                with torch.cuda.stream(cs):
                    cg.replay()
                torch.cuda.synchronize()
            else:
                with torch.cuda.stream(cs):
                    b.update_factors()
        torch.cuda.synchronize()
        assert b.sync_streams() == 0
    else:
        for t in range(nsteps):
            with torch.cuda.stream(cs):
                for i, st in enumerate(streams):
                    Xb[i].copy_(torch.from_numpy(data[t][i][0]))
                    Sb[i].copy_(torch.from_numpy(data[t][i][1]))
                    st.update_factors(Xb[i], Sb[i])
        torch.cuda.synchronize()
    infos = [st.info() for st in streams]
    if kappa_f:
        for st, inf in zip(streams, infos):
            inf["fac"] = st.factor_info()
    return [[a.cpu().numpy() for a in st.factors()] for st in streams], infos


def test_batch_steps_match_per_stream_steps():
    print("case: batch steps", flush=True)
    ref_f, ref_i = _run_steps(False, False)
    got_f, got_i = _run_steps(True, False)
    for i in range(len(SPECS)):
        assert got_i[i]["t"] == ref_i[i]["t"] and got_i[i]["slot_times"] == ref_i[i]["slot_times"]
        assert got_i[i]["adam_iter"] == ref_i[i]["adam_iter"]
        for k in range(3):
            assert rel_err(got_f[i][k], ref_f[i][k]) <= 1e-6, (i, k)


def test_batch_graph_replay_matches_eager():
    """One time step captured as a HIP graph, replayed with new inputs copied
    in between replays, equals the eager batched steps."""
    print("case: batch graph", flush=True)
    eager_f, eager_i = _run_steps(True, False)
    graph_f, graph_i = _run_steps(True, True)
    for i in range(len(SPECS)):
        assert graph_i[i]["slot_times"] == eager_i[i]["slot_times"]
        for k in range(3):
            assert np.array_equal(graph_f[i][k], eager_f[i][k]), (i, k)


def test_batch_solve_st_matches_streams_and_oracle():
    """Batched LS temporal solve: Gaussian streams get the per-stream result
    (same kernels, same inputs: bitwise) and the oracle's within tolerance;
    other streams keep the s_t their caller wrote."""
    import torch
    from oracle.solve import ls_temporal
    from paper_2110_14514_amd import Batch
    print("case: batch solve_st", flush=True)
    probs = _problems()
    devs, streams = _make(probs)
    Xb = [d["X_t"].clone() for d in devs]
    Sb = [d["s_t"].clone() for d in devs]
    before = [s.clone() for s in Sb]
    b = Batch(streams, Xb, Sb)
    b.solve_st()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    n_gauss = 0
    for i, (p, d, st) in enumerate(zip(probs, devs, streams)):
        if p.loss != "gaussian":
            assert torch.equal(Sb[i], before[i]), i
            continue
        n_gauss += 1
        ref = st.solve_st(d["X_t"])
        torch.cuda.synchronize()
        assert torch.equal(Sb[i], ref), i
        pp = p.promoted()
        assert rel_err(Sb[i].double().cpu().numpy(), ls_temporal(pp.X_t, pp.A, p.mu)) <= TOL, i
    assert n_gauss >= 2


def test_batch_autotune_matches_oracle(tmp_path):
    """gcp_batch_autotune times batched calls over the candidate plans and
    gives every stream the fastest; the batch built on the tuned plan
    (launches spread over its lanes) still matches the oracle, and a second
    tuning of the same shape buckets reads the plan from the cache."""
    import torch
    from paper_2110_14514_amd import Batch
    print("case: batch autotune", flush=True)
    probs = _problems() + [gi.random_dense((22, 18, 70), 16, 4, "gaussian", seed=41, lam=0.05, mu=0.1)]
    devs, streams = _make(probs)
    cache = tmp_path / "tune.txt"
    b = Batch(streams, [d["X_t"].clone() for d in devs], [d["s_t"].clone() for d in devs],
              autotune=True, tune_cache=str(cache))
    assert 1 <= b.buckets < len(probs)          # the two rank-16 Gaussian streams share a bucket
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and f"buckets{b.buckets} " in lines[0]
    assert int(lines[0].rsplit("=", 1)[1]) in (512, 1024, 2048, 4096)
    outs = b.loss_grad()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    for i, p in enumerate(probs):
        bl, bG, bg = outs[i]
        got = (float(bl.item()), [g.double().cpu().numpy() for g in bG], bg.double().cpu().numpy())
        errs = compare(p, got, og)
        assert max(errs.values()) <= TOL, (i, errs)
    devs2, streams2 = _make(probs)
    b2 = Batch(streams2, [d["X_t"].clone() for d in devs2], [d["s_t"].clone() for d in devs2],
               autotune=True, tune_cache=str(cache))
    assert b2.buckets == b.buckets and cache.read_text().splitlines() == lines


def test_batch_epochs_match_per_stream_epochs():
    """kappa_f = 2 epochs of tau_f = 2 steps per time step in a batch: the
    same keep/undo decisions, rates, objectives and factors as each stream's
    own gcp_update_factors (which the oracle pins)."""
    print("case: batch epochs", flush=True)
    ref_f, ref_i = _run_steps(False, False, kappa_f=2)
    got_f, got_i = _run_steps(True, False, kappa_f=2)
    for i in range(len(SPECS)):
        assert got_i[i]["t"] == ref_i[i]["t"] and got_i[i]["slot_times"] == ref_i[i]["slot_times"]
        gf, rf = got_i[i]["fac"], ref_i[i]["fac"]
        assert gf["rolled"] == rf["rolled"] and gf["epochs"] == rf["epochs"] and gf["iters"] == rf["iters"], (i, gf, rf)
        assert gf["alpha"] == rf["alpha"], i
        assert abs(gf["F"] - rf["F"]) <= 1e-6 * abs(rf["F"]), (i, gf["F"], rf["F"])
        for k in range(3):
            assert rel_err(got_f[i][k], ref_f[i][k]) <= 1e-5, (i, k)


def test_batch_epochs_graph_replay_matches_eager():
    """A time step with epochs captured once as a HIP graph and replayed
    equals the eager batched steps bit for bit, decisions included."""
    print("case: batch epochs graph", flush=True)
    eager_f, eager_i = _run_steps(True, False, kappa_f=2)
    graph_f, graph_i = _run_steps(True, True, kappa_f=2)
    for i in range(len(SPECS)):
        assert graph_i[i]["slot_times"] == eager_i[i]["slot_times"]
        assert graph_i[i]["fac"] == eager_i[i]["fac"], i
        for k in range(3):
            assert np.array_equal(graph_f[i][k], eager_f[i][k]), (i, k)



# window capacity H against slices held: two-h-tile builds (H >= 16) whose
# windows still hold at most 16 slices, and one-h-tile windows of 9..15
# slices (the last h-tile's GEMM2 K-steps fixed per work item at 3 and 4)
FILL_SPECS = [((21, 13, 37), 16, 20, 9, "gaussian"), ((17, 11, 44), 32, 24, 14, "poisson_log"),
              ((19, 15, 52), 16, 10, 10, "poisson_log"), ((13, 22, 48), 32, 14, 14, "gaussian"),
              ((25, 9, 61), 8, 12, 12, "gaussian"), ((11, 14, 36), 32, 9, 9, "poisson_log")]


def test_batch_partial_and_mid_windows_match_streams_and_oracle():
    import torch
    from paper_2110_14514_amd import Batch, Stream
    print("case: batch partial / mid windows", flush=True)
    probs = [gi.random_dense(d, R, n, loss, seed=40 + i, w=1.1, theta=0.9, lam=0.05, mu=0.1)
             for i, (d, R, H, n, loss) in enumerate(FILL_SPECS)]
    devs = [to_device(p) for p in probs]
    streams = [Stream(p.dims, p.rank, H, p.loss, d["A"], d["X_hist"], d["s_hist"], d["t_hist"], w=p.w,
                      theta=p.theta, lam=p.lam, mu=p.mu, kernel="mfma")
               for p, d, (_, _, H, _, _) in zip(probs, devs, FILL_SPECS)]
    b = Batch(streams, [d["X_t"].clone() for d in devs], [d["s_t"].clone() for d in devs])
    outs = b.loss_grad()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    for i, (p, d, st) in enumerate(zip(probs, devs, streams)):
        loss, G, g_s = st.loss_grad(d["X_t"], d["A"], d["s_t"])
        torch.cuda.synchronize()
        bl, bG, bg = outs[i]
        # the batch's build has the window's capacity in h-tiles, the
        # stream's own call the slices it holds: same sums up to their order
        assert rel_err(bl.cpu().numpy(), loss.cpu().numpy()) <= 1e-5, i
        for k in range(3):
            assert rel_err(bG[k].cpu().numpy(), G[k].cpu().numpy()) <= 1e-5, (i, k)
        assert rel_err(bg.cpu().numpy(), g_s.cpu().numpy()) <= 1e-5, i
        got = (float(bl.item()), [g.double().cpu().numpy() for g in bG], bg.double().cpu().numpy())
        errs = compare(p, got, og)
        assert max(errs.values()) <= TOL, (i, errs)
