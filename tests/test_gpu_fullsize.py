"""Parity at the full sizes of the benchmarked configurations, in the launch
configuration the benchmark times, against the FP64 oracle.

Where the oracle cannot evaluate the whole gradient in seconds it checks
sampled outputs one by one: row r of G^(k) is the mode-k gradient of the
sub-problem whose slices are restricted to the slab i_k = r (every term of
row r lives in that slab), and g_s is the sum of the g_s of row slabs of
X_t (the model and the loss derivative are entrywise, so the sum over slabs
is the sum over the slice).  Every comparison is normwise and per element
against the column's largest reference value.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle import sampled as osm

from helpers import TOL, compare, elem_err, grad_err, loss_err, make_stream, rel_err, to_device

pytestmark = pytest.mark.gpu


def _case(*a):
    print("case:", *a, flush=True)


def _host(x):
    return x.double().cpu().numpy()


def _sub(prob, k, lo, hi):
    """The problem restricted to the slab lo <= i_k < hi (slices and A^(k))."""
    cut = lambda X: np.take(X, np.arange(lo, hi), axis=k)
    A = list(prob.A)
    A[k] = A[k][lo:hi]
    return SimpleNamespace(X_t=cut(prob.X_t), A=A, s_t=prob.s_t, X_hist=[cut(x) for x in prob.X_hist],
                           s_hist=prob.s_hist, t_hist=prob.t_hist, t=prob.t, w=prob.w, theta=prob.theta,
                           lam=prob.lam, mu=prob.mu, loss=prob.loss)


def oracle_row(prob, k, r):
    G, _ = og.gradient(_sub(prob, k, r, r + 1))
    return G[k][0]


def oracle_gs(prob, slab=16):
    """g_s from row slabs of X_t (no window term, Q4), mu s_t added once."""
    I1 = prob.X_t.shape[0]
    gs = np.zeros(len(prob.s_t))
    for lo in range(0, I1, slab):
        sub = _sub(prob, 0, lo, min(I1, lo + slab))
        sub.X_hist, sub.s_hist, sub.t_hist, sub.mu = [], np.zeros((0, len(prob.s_t))), [], 0.0
        gs += og.gradient(sub)[1]
    return gs + prob.mu * np.asarray(prob.s_t, np.float64)


def check_rows(prob, G, g_s, rows):
    """Sampled rows of every G^(k) and the whole g_s against the oracle; each
    row is compared per element against its columns' largest values over the
    sampled rows."""
    for k in range(3):
        ref = np.stack([oracle_row(prob, k, r) for r in rows[k]])
        got = np.stack([G[k][r] for r in rows[k]])
        assert grad_err(got, ref) <= TOL, (k, rows[k], rel_err(got, ref), elem_err(got, ref))
    gsr = oracle_gs(prob)
    assert grad_err(g_s, gsr) <= TOL, (rel_err(g_s, gsr), elem_err(g_s, gsr))


def _host_problem(dims, R, loss, X_t, A, s_t, Xh, Sh, **kw):
    H = len(Xh)
    return SimpleNamespace(dims=tuple(dims), rank=R, X_t=_host(X_t), A=[_host(a) for a in A], s_t=_host(s_t),
                           X_hist=[_host(x) for x in Xh], s_hist=_host(Sh) if H else np.zeros((0, R)),
                           t_hist=np.arange(1, H + 1), t=H + 1, w=kw.get("w", 1.0), theta=kw.get("theta", 1.0),
                           lam=kw.get("lam", 0.0), mu=kw.get("mu", 0.0), loss=loss)


def test_c3_full_size_sampled_rows():
    """C3: 1000 x 1000 x 64 binary slices, rank 32, window 20, Bernoulli-logit,
    the benchmark's inputs and call (FP32 matrix-core kernel with two h-tiles
    and 16-byte copies); three rows of each G^(k), all of g_s."""
    import torch
    from paper_2110_14514_amd import Stream
    _case("C3 full size")
    dims, R, H, loss = (1000, 1000, 64), 32, 20, "bernoulli_logit"
    X_t, A, s_t, Xh, Sh = gi.device_dense_window(dims, R, H, loss, seed=2)
    st = Stream(dims, R, H, loss, A, Xh, Sh, list(range(1, H + 1)))
    out = (torch.empty(1, device="cuda"), [torch.empty(n, R, device="cuda") for n in dims],
           torch.empty(R, device="cuda"))
    st.loss_grad(X_t, A, s_t, out=out)
    torch.cuda.synchronize()
    assert st.sync() == 0
    G = [_host(g) for g in out[1]]
    g_s = _host(out[2])
    del st
    prob = _host_problem(dims, R, loss, X_t, A, s_t, Xh, Sh)
    check_rows(prob, G, g_s, [[0, 517, 999], [1, 333, 998], [0, 31, 63]])


def test_c3_shaped_sub_instance_all_outputs_through_autograd():
    """C3's kernel build (rank tile 32, two h-tiles, 64-wide I3) at 320 x 320 x
    64 (102,400 (i1, i2) pairs feeding every G^(3) row, as C3's million do in
    kind): the FP32 autograd path's objective and every gradient output."""
    import torch
    from paper_2110_14514_amd import gcp_loss
    _case("C3 sub-instance autograd")
    prob = gi.c3_problem(dims=(320, 320, 64))
    dev = to_device(prob)
    st = make_stream(prob, dev, kernel="mfma")
    A = [a.clone().requires_grad_(True) for a in dev["A"]]
    s = dev["s_t"].clone().requires_grad_(True)
    F = gcp_loss(st, dev["X_t"], A, s)
    F.backward()
    torch.cuda.synchronize()
    assert st.sync() == 0
    got = (float(F.item()), [_host(a.grad) for a in A], _host(s.grad))
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


def _variant(loss, R, H, I3):
    """The batched path's tile class of a stream: loss, rank tile, h-tiles and
    copy width (used here only to pick one stream of each class)."""
    return (loss, R > 16, H + 1 > 16, I3 % 4 == 0)


def test_c4_full_batch_against_oracle():
    """C4: the 64-stream batch exactly as benchmarked (dims U{50..300}^3,
    ranks {8,16,32}, windows 4..16, Gaussian/Poisson-log); the smallest
    stream of every tile class is checked in full (objective and every
    output), the largest stream of the batch by sampled rows and g_s."""
    import torch
    from paper_2110_14514_amd import Batch, Stream
    _case("C4 batch full size")
    specs = gi.c4_specs()
    streams, Xb, Sb, data = [], [], [], []
    for sp in specs:
        X_t, A, s_t, Xh, Sh = gi.device_dense_window(sp.dims, sp.rank, sp.window, sp.loss, sp.seed)
        streams.append(Stream(sp.dims, sp.rank, sp.window, sp.loss, A, Xh, Sh, list(range(1, sp.window + 1)),
                              alpha_f=1e-4, tau_f=1))
        Xb.append(X_t)
        Sb.append(s_t)
        data.append((A, Xh, Sh))
    torch.cuda.synchronize()
    b = Batch(streams, Xb, Sb)
    outs = b.loss_grad()
    torch.cuda.synchronize()
    assert b.sync_streams() == 0
    classes = {}
    for i, sp in enumerate(specs):
        key = _variant(sp.loss, sp.rank, sp.window, sp.dims[2])
        om = int(np.prod(sp.dims))
        if key not in classes or om < classes[key][0]:
            classes[key] = (om, i)
    full = sorted(i for _, i in classes.values())
    big = int(np.argmax([np.prod(sp.dims) * (sp.window + 1) for sp in specs]))
    _case("C4 full checks on streams", full, "rows on stream", big)
    for i in full + [big]:
        sp = specs[i]
        A, Xh, Sh = data[i]
        prob = _host_problem(sp.dims, sp.rank, sp.loss, Xb[i], A, Sb[i], Xh, Sh)
        loss, G, g_s = outs[i]
        G = [_host(g) for g in G]
        g_s = _host(g_s)
        if i in full and np.prod(sp.dims) <= 4_000_000:
            F = og.objective(prob)
            assert loss_err(loss.item(), F, og.loss_terms_abs(prob)) <= TOL, (i, sp)
            Gr, gsr = og.gradient(prob)
            for k in range(3):
                assert grad_err(G[k], Gr[k]) <= TOL, (i, sp, k, rel_err(G[k], Gr[k]), elem_err(G[k], Gr[k]))
            assert grad_err(g_s, gsr) <= TOL, (i, sp)
        else:
            rows = [[0, d // 2, d - 1] for d in sp.dims]
            check_rows(prob, G, g_s, rows)


def test_c5_full_size_slice_against_regenerated_draws():
    """C5's slice at full size: 2000 x 2000 x 500 COO with 2M nonzeros, rank
    32, p = q = 2M draws (no window), Poisson-log; the oracle regenerates the
    same 4M Philox draws and forms the objective and every output."""
    import torch
    from paper_2110_14514_amd import Stream
    _case("C5 full-size slice")
    prob = gi.sparse_problem(window=0)
    T = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    st = Stream(prob.dims, prob.rank, 0, prob.loss, [T(a) for a in prob.A], [], None, [], seed=prob.seed,
                slice_kind="coo", max_nnz=prob.X_t.coords.shape[0], p=prob.p, q=prob.q)
    loss, G, g_s = st.loss_grad((T(prob.X_t.coords, torch.int32), T(prob.X_t.vals)), [T(a) for a in prob.A],
                                T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    prob.A = [a.astype(np.float32).astype(np.float64) for a in prob.A]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    F, Gr, gsr = osm.sampled_loss_grad(prob, call=0)
    assert abs(float(loss.item()) - F) / abs(F) <= TOL
    for k in range(3):
        got = _host(G[k])
        assert grad_err(got, Gr[k]) <= TOL, (k, rel_err(got, Gr[k]), elem_err(got, Gr[k]))
    assert grad_err(_host(g_s), gsr) <= TOL


def test_c5_benchmark_call_weight_gradient():
    """C5 as benchmarked (window of 8 stored COO slices, 36M draws per call,
    the launch configuration of that draw count): g_s depends on X_t's draws
    alone, which the oracle regenerates."""
    import torch
    from paper_2110_14514_amd import Stream
    _case("C5 benchmark call, g_s")
    prob = gi.sparse_problem()
    T = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    coo = lambda sl: (T(sl.coords, torch.int32), T(sl.vals))
    H = len(prob.X_hist)
    st = Stream(prob.dims, prob.rank, H, prob.loss, [T(a) for a in prob.A], [coo(x) for x in prob.X_hist],
                T(prob.s_hist), list(prob.t_hist), seed=prob.seed, slice_kind="coo",
                max_nnz=prob.X_t.coords.shape[0], p=prob.p, q=prob.q)
    loss, G, g_s = st.loss_grad(coo(prob.X_t), [T(a) for a in prob.A], T(prob.s_t))
    torch.cuda.synchronize()
    assert st.sync() == 0
    prob.A = [a.astype(np.float32).astype(np.float64) for a in prob.A]
    prob.s_t = prob.s_t.astype(np.float32).astype(np.float64)
    prob.X_hist, prob.s_hist, prob.t_hist = [], np.zeros((0, prob.rank)), np.zeros(0, np.int64)
    _, _, gsr = osm.sampled_loss_grad(prob, call=0)
    assert grad_err(_host(g_s), gsr) <= TOL


def test_e5_shape_window_50():
    """The paper's synthetic Gaussian shape: 300 x 300 matrix slices, rank 20,
    window 50, every dense kernel, against the two-way oracle."""
    import torch
    from oracle.stream import StreamOracle
    from paper_2110_14514_amd import Stream
    _case("E5 shape window 50")
    dims, R, H = (300, 300), 20, 50
    g = np.random.default_rng(55)
    A = [g.uniform(-0.5, 0.5, (n, R)).astype(np.float32) for n in dims]
    Xs = [g.normal(size=dims).astype(np.float32) for _ in range(H + 1)]
    S = g.uniform(0.5, 1.5, (H + 1, R)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    kw = dict(w=1.0, theta=0.97, lam=0.01, mu=0.02)
    orc = StreamOracle([a.astype(np.float64) for a in A], [x.astype(np.float64) for x in Xs[1:]],
                       S[1:].astype(np.float64), list(range(1, H + 1)), loss="gaussian", window=H, d=2, **kw)
    X64 = Xs[0].astype(np.float64)
    s64 = S[0].astype(np.float64)
    p = orc.problem(X64.reshape(dims + (1,)), s64)
    Gr, gsr = og.gradient(p)
    F = orc.factor_objective(X64, s64) + 0.5 * kw["mu"] * float(s64 @ s64)
    scale = og.loss_terms_abs(p)
    for kernel in ("valu", "mfma", "auto"):
        st = Stream(dims, R, H, "gaussian", [T(a) for a in A], [T(x) for x in Xs[1:]], T(S[1:]),
                    list(range(1, H + 1)), kernel=kernel, **kw)
        loss, G, gs = st.loss_grad(T(Xs[0]), [T(a) for a in A], T(S[0]))
        torch.cuda.synchronize()
        assert st.sync() == 0
        assert loss_err(loss.item(), F, scale) <= TOL, kernel
        for k in range(2):
            assert grad_err(_host(G[k]), Gr[k]) <= TOL, (kernel, k)
        assert grad_err(_host(gs), gsr) <= TOL, kernel
