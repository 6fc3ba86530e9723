"""GPU parity of the dense path (fused and unfused) against the FP64 oracle,
through the C ABI.  Normwise relative tolerance 1e-5 on FP32 results."""
import math
import zlib

import numpy as np
import pytest

import gcp_inputs as gi
from oracle import gcp as og
from oracle.solve import ls_temporal
from oracle.stream import StreamOracle

from helpers import TOL, compare, gpu_loss_grad, make_stream, rel_err, to_device

pytestmark = pytest.mark.gpu

# (dims, rank, window): several tiles, ragged pair tiles, ragged i3 chunks
# (I3 not a multiple of 64), ranks that are not a power of two, R = 64.
SHAPES = [
    ((5, 6, 7), 4, 0),
    ((7, 9, 70), 5, 2),
    ((17, 33, 129), 16, 3),
    ((9, 4, 64), 32, 1),
    ((20, 30, 40), 8, 10),
    ((3, 3, 3), 64, 1),
    ((40, 41, 13), 12, 4),
    ((6, 5, 200), 16, 20),      # two h-tiles, 3 full 64-wide groups + 8-wide tail
    ((4, 7, 66), 32, 40),       # three h-tiles, I3 not a multiple of 4
    ((3, 4, 128), 20, 60),      # four h-tiles
    ((9, 10, 48), 16, 4),       # 32-wide group + 16-wide tail (one-tile tail)
    ((11, 13, 52), 16, 6),      # 32-wide group + 20-wide tail (two-tile tail)
    ((12, 10, 64), 32, 20),     # C3's build: rank tile 32, two h-tiles, 16-byte copies
    ((8, 9, 68), 24, 24),       # the same build at rank 24, 25 slices, a 4-wide tail
    ((7, 5, 33), 16, 7),        # two pairs per step, 8 slices, odd pair count, 4-byte copies
    ((13, 11, 96), 32, 5),      # two pairs per step at rank tile 32, 16-byte copies
    ((9, 7, 45), 32, 6),        # rank tile 32, two pairs per step, odd pair count, 4-byte copies, 13-wide tail
    ((15, 11, 100), 24, 12),    # rank tile 32, one h-tile with four registers of slices, 16-byte copies
    ((5, 3, 70), 32, 9),        # 15 pairs: most waves of the four-wave workgroups hold no block
    ((6, 7, 99), 32, 20),       # two h-tiles at rank tile 32, stored rows by 16-byte copies, I3 not a multiple of 4
    ((5, 9, 101), 16, 18),      # two h-tiles at rank tile 16, the same copy mode
]


def _print_case(*a):
    print("case:", *a, flush=True)


@pytest.mark.parametrize("kernel", ["valu", "mfma"])
@pytest.mark.parametrize("loss", og.LOSSES)
@pytest.mark.parametrize("dims,R,H", SHAPES)
def test_fused_matches_oracle(dims, R, H, loss, kernel):
    _print_case("fused", kernel, dims, R, H, loss)
    prob = gi.random_dense(dims, R, H, loss, seed=zlib.crc32(repr((dims, R, H, loss)).encode()) % 1000,
                           w=1.3, theta=0.8, lam=0.05, mu=0.2)
    got, code, _ = gpu_loss_grad(prob, kernel=kernel)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("loss", og.LOSSES)
@pytest.mark.parametrize("dims,R,H", SHAPES[:5])
def test_plain_matches_oracle(dims, R, H, loss):
    _print_case("plain", dims, R, H, loss)
    prob = gi.random_dense(dims, R, H, loss, seed=17, w=0.7, theta=0.9, lam=0.1, mu=0.05)
    got, code, _ = gpu_loss_grad(prob, plain=True)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("loss", og.LOSSES)
def test_fp64_instantiation_is_exact(loss):
    _print_case("fp64", loss)
    prob = gi.random_dense((6, 7, 67), 6, 2, loss, seed=3, w=1.1, theta=0.7, lam=0.2,
                           mu=0.3, dtype=np.float64)
    got, code, _ = gpu_loss_grad(prob)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= 1e-12, errs


def test_c1_config():
    _print_case("C1")
    prob = gi.c1_problem()
    got, code, _ = gpu_loss_grad(prob)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("kernel", ["auto", "valu"])
def test_c2_full_size(kernel):
    """C2 at its full size (200^3, R=16, H=10, Poisson-log) in the launch
    configuration the bench times (automatic kernel choice); every output
    compared."""
    _print_case("C2 full", kernel)
    prob = gi.c2_problem()
    got, code, _ = gpu_loss_grad(prob, kernel=kernel)
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


def test_bitwise_repeatable():
    import torch
    _print_case("repeat")
    prob = gi.random_dense((17, 33, 129), 16, 3, "poisson_log", seed=5)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    outs = []
    for _ in range(3):
        loss, G, g_s = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
        torch.cuda.synchronize()
        outs.append([loss.cpu().numpy()] + [g.cpu().numpy() for g in G] + [g_s.cpu().numpy()])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_want_loss_only_and_grad_only():
    import torch
    _print_case("want bits")
    prob = gi.random_dense((8, 9, 10), 4, 2, "bernoulli_logit", seed=6)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    l1, G1, g1 = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    G = [torch.full_like(g, 7.0) for g in G1]
    gs = torch.full_like(g1, 7.0)
    loss = torch.full_like(l1, 7.0)
    st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], want_grad=False, out=(loss, G, gs))
    torch.cuda.synchronize()
    assert loss.item() == l1.item()
    assert all(torch.all(g == 7.0) for g in G) and torch.all(gs == 7.0)
    loss.fill_(7.0)
    st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], want_loss=False, out=(loss, G, gs))
    torch.cuda.synchronize()
    assert loss.item() == 7.0 and torch.equal(G[0], G1[0]) and torch.equal(gs, g1)


def test_nonfinite_is_reported():
    import torch
    _print_case("nonfinite")
    prob = gi.random_dense((8, 9, 10), 4, 0, "poisson_log", seed=7)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    dev["X_t"][1, 2, 3] = float("nan")
    st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    assert st.sync() == 7          # GCP_E_NUMERIC, then cleared
    dev["X_t"][1, 2, 3] = 0.0
    st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    assert st.sync() == 0


def test_ls_solve_matches_oracle():
    import torch
    _print_case("ls solve")
    for dims, R, mu in [((20, 30, 40), 4, 0.0), ((33, 17, 129), 16, 0.5), ((9, 10, 11), 32, 1.0)]:
        prob = gi.random_dense(dims, R, 0, "gaussian", seed=R)
        prob.mu = mu
        dev = to_device(prob)
        st = make_stream(prob, dev)
        s = st.solve_st(dev["X_t"])
        torch.cuda.synchronize()
        assert st.sync() == 0
        ref = ls_temporal(prob.promoted().X_t, prob.promoted().A, mu)
        assert rel_err(s.cpu().numpy(), ref) <= TOL


def test_singular_gram_is_reported():
    import torch
    _print_case("singular")
    prob = gi.random_dense((6, 7, 8), 3, 0, "gaussian", seed=2)
    prob.A[0][:, 2] = 0.0          # Gamma singular with mu = 0
    dev = to_device(prob)
    st = make_stream(prob, dev)
    s = st.solve_st(dev["X_t"])
    torch.cuda.synchronize()
    assert st.sync() == 7
    assert torch.isnan(s).all()


def test_stream_steps_match_oracle():
    """C1 stream: five OnlineGCP steps (LS weights, tau_f=3 Adam iterations
    with window, reservoir push) against the oracle stream."""
    import torch
    _print_case("stream C1")
    data = gi.c1_stream()
    H = 3
    g = gi.rng(99)
    A0 = [a + 0.1 * g.standard_normal(a.shape) for a in data.A_true]
    Xf = data.X.astype(np.float32)
    A0f = [a.astype(np.float32) for a in A0]
    S0 = data.S_true[:H].astype(np.float32)
    kw = dict(loss="gaussian", window=H, w=1.0, theta=0.95, lam=0.01, mu=0.02,
              alpha_f=1e-2, tau_f=3, seed=11)
    orc = StreamOracle([a.astype(np.float64) for a in A0f], [x.astype(np.float64) for x in Xf[:H]],
                       S0.astype(np.float64), np.arange(1, H + 1), **kw)
    from paper_2110_14514_amd import Stream
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(Xf.shape[1:], 4, H, "gaussian", [tt(a) for a in A0f], [tt(x) for x in Xf[:H]],
                tt(S0), list(range(1, H + 1)), w=1.0, theta=0.95, lam=0.01, mu=0.02,
                alpha_f=1e-2, tau_f=3, seed=11)
    for t in range(H, H + 8):
        X = tt(Xf[t])
        s_gpu = st.step(X)
        s_or = orc.step(Xf[t].astype(np.float64))
        torch.cuda.synchronize()
        assert st.sync() == 0
        assert rel_err(s_gpu.cpu().numpy(), s_or) <= 1e-4
        info = st.info()
        assert info["t"] == orc.t and info["slot_times"] == orc.slots
    A_gpu = [a.cpu().numpy() for a in st.factors()]
    for k in range(3):
        assert rel_err(A_gpu[k], orc.A[k]) <= 1e-4
        assert rel_err(A_gpu[k] - A0f[k], orc.A[k] - A0f[k]) <= 1e-2


def _tune_key(st, prob, ns):
    """The autotuner's shape bucket: tile build, pair count by powers of two,
    I3 by 64-entry groups.  A stream's stored rows are padded to 32 values,
    so its copy mode is 2 when I3 is a multiple of 4, else 1."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    loss_id = {"gaussian": 0, "poisson_log": 1, "bernoulli_logit": 2}[prob.loss]
    d = prob.dims
    lp = (d[0] * d[1]).bit_length() - 1
    return (f"{arch} loss{loss_id} rt{32 if prob.rank > 16 else 16} nh{(ns + 15) // 16} "
            f"dma{2 if d[2] % 4 == 0 else 1} pairs2^{lp} i3x64:{(d[2] + 63) // 64}")


@pytest.mark.parametrize("target", [1024, 2048, 4096, 8192, 16384])
def test_every_autotune_candidate_matches_oracle(target, tmp_path):
    """Each candidate work plan (forced through the cache) gives the oracle's
    result: the plan changes only the summation order."""
    import torch
    _print_case("plan", target)
    prob = gi.random_dense((37, 45, 70), 16, 3, "poisson_log", seed=31, lam=0.1, mu=0.1)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{_tune_key(st, prob, 4)} = {target}\n")
    assert st.autotune(dev["X_t"], str(cache)) == target
    loss, G, g_s = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
    got = (float(loss.item()), [g.double().cpu().numpy() for g in G], g_s.double().cpu().numpy())
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


def test_autotune_writes_and_reuses_cache(tmp_path):
    import torch
    _print_case("autotune cache")
    prob = gi.random_dense((64, 64, 64), 16, 5, "gaussian", seed=32)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    cache = tmp_path / "tune.txt"
    chosen = st.autotune(dev["X_t"], str(cache))
    assert chosen in (1024, 2048, 4096, 8192, 16384)
    text = cache.read_text()
    assert _tune_key(st, prob, 6) in text and text.strip().endswith(str(chosen))
    st2 = make_stream(prob, dev)
    assert st2.autotune(dev["X_t"], str(cache)) == chosen
    assert cache.read_text() == text      # a hit appends nothing
    # a stream of another shape in the same bucket takes the cached plan
    prob3 = gi.random_dense((60, 70, 60), 16, 5, "gaussian", seed=33)
    dev3 = to_device(prob3)
    st3 = make_stream(prob3, dev3)
    assert _tune_key(st3, prob3, 6) == _tune_key(st, prob, 6)
    assert st3.autotune(dev3["X_t"], str(cache)) == chosen and cache.read_text() == text
    # a value that is not a candidate plan is not taken from the cache
    cache.write_text(f"{_tune_key(st, prob, 6)} = 777\n")
    assert st2.autotune(dev["X_t"], str(cache)) in (1024, 2048, 4096, 8192, 16384)


# One slice and no window: the pairs-in-rows matrix-core kernel.  Ragged
# 4 x 4 pair blocks (I1, I2 not multiples of 4), I3 odd or not a multiple of
# 32, a single entry, ranks below, at and between the 16 / 32 tiles.
SINGLE = [((5, 6, 7), 4), ((9, 7, 33), 16), ((13, 11, 64), 32), ((4, 4, 1), 20), ((17, 3, 45), 5),
          ((1, 1, 100), 32), ((30, 41, 200), 16), ((2, 9, 31), 12)]


@pytest.mark.parametrize("loss", og.LOSSES)
@pytest.mark.parametrize("dims,R", SINGLE)
def test_single_slice_matches_oracle(dims, R, loss):
    _print_case("single slice", dims, R, loss)
    prob = gi.random_dense(dims, R, 0, loss, seed=zlib.crc32(repr((dims, R, loss)).encode()) % 1000,
                           lam=0.05, mu=0.2)
    got, code, _ = gpu_loss_grad(prob, kernel="auto")
    assert code == 0
    errs = compare(prob, got, og)
    assert max(errs.values()) <= TOL, errs


def test_single_slice_is_bitwise_repeatable():
    import torch
    _print_case("single slice repeat")
    prob = gi.random_dense((37, 29, 70), 16, 0, "poisson_log", seed=5)
    dev = to_device(prob)
    st = make_stream(prob, dev)
    a = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    a = (a[0].clone(), [g.clone() for g in a[1]], a[2].clone())
    b = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and all(torch.equal(x, y) for x, y in zip(a[1], b[1])) and torch.equal(a[2], b[2])
