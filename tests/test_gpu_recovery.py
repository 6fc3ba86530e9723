"""Planted recovery through the library: the C1 Gaussian stream and a small
Poisson-log count stream (temporal weights by Algorithm 3, factor epochs of
Algorithm 4) run step by step through the C ABI beside the oracle stream,
whose own recovery is pinned in test_oracle_recovery.py.  Each step compares
s_t, and the run compares the factors, the local loss of eq. `local_loss`
and the K-tensor score of Section 6.1 computed by the library with the
oracle's, and checks the recovery thresholds on the library's own metrics."""
import numpy as np
import pytest

import gcp_inputs as gi
from oracle.metrics import ktensor_score, local_loss, slice_loss
from oracle.stream import StreamOracle

from helpers import rel_err
from test_oracle_recovery import C1_H, POIS_H, c1_start, deviance, noise_floor, poisson_start

pytestmark = pytest.mark.gpu


def test_c1_stream_recovery_matches_oracle():
    import torch
    from paper_2110_14514_amd import Stream
    print("case: C1 planted recovery, FP32, 17 steps", flush=True)
    data, A0, S0 = c1_start()
    Xf = data.X.astype(np.float32)
    A0f = [a.astype(np.float32) for a in A0]
    S0f = S0.astype(np.float32)
    kw = dict(alpha_f=1e-2, tau_f=20, seed=0)
    orc = StreamOracle([a.astype(np.float64) for a in A0f], [x.astype(np.float64) for x in Xf[:C1_H]],
                       S0f.astype(np.float64), np.arange(1, C1_H + 1), loss="gaussian", window=C1_H, **kw)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = Stream(Xf.shape[1:], 4, C1_H, "gaussian", [T(a) for a in A0f], [T(x) for x in Xf[:C1_H]], T(S0f),
                list(range(1, C1_H + 1)), **kw)
    B = [T(a.astype(np.float32)) for a in data.A_true]
    for t in range(C1_H, Xf.shape[0]):
        X = T(Xf[t])
        s_gpu = st.step(X)
        s_or = orc.step(Xf[t].astype(np.float64))
        torch.cuda.synchronize()
        assert st.sync() == 0
        assert rel_err(s_gpu.cpu().numpy(), s_or) <= 1e-4, t
        ll_gpu = st.local_loss(X, s_gpu)
        ll_or = local_loss(Xf[t].astype(np.float64), orc.A, s_or, "gaussian")
        assert abs(ll_gpu - ll_or) <= 1e-4 * ll_or, (t, ll_gpu, ll_or)
        sc_gpu = st.ktensor_score(s_gpu, B, T(data.S_true[t].astype(np.float32)))
        sc_or = ktensor_score(orc.A, s_or, data.A_true, data.S_true[t])
        assert abs(sc_gpu - sc_or) <= 1e-4, (t, sc_gpu, sc_or)
        if t >= C1_H + 4:
            assert 0.97 <= ll_gpu / noise_floor(data, t) <= 1.01, t
            assert sc_gpu >= 0.997, t
    A_gpu = [a.cpu().numpy() for a in st.factors()]
    for k in range(3):
        assert rel_err(A_gpu[k], orc.A[k]) <= 1e-4


def test_poisson_stream_recovery_with_both_sgd_solvers_matches_oracle():
    """FP64 on the device, so that every epoch decision of both solvers is
    taken on the same values as the oracle's."""
    import torch
    from paper_2110_14514_amd import Stream
    print("case: Poisson planted recovery, FP64, weight SGD + factor epochs", flush=True)
    data, A0, S0, _ = poisson_start()
    kw = dict(alpha_f=1e-2, tau_f=20, kappa_f=5, seed=3, tsolve="sgd", tau_w=100, kappa_w=20, alpha_w=1.0)
    orc = StreamOracle(A0, [data.X[h] for h in range(POIS_H)], S0, np.arange(1, POIS_H + 1),
                       loss="poisson_log", window=POIS_H, **kw)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    st = Stream(data.X.shape[1:], 3, POIS_H, "poisson_log", [T(a) for a in A0],
                [T(data.X[h]) for h in range(POIS_H)], T(S0), list(range(1, POIS_H + 1)), **kw)
    B = [T(a) for a in data.A_true]
    for t in range(POIS_H, data.X.shape[0]):
        X = T(data.X[t])
        s_gpu = st.step(X)
        s_or = orc.step(data.X[t])
        torch.cuda.synchronize()
        assert st.sync() == 0
        assert rel_err(s_gpu.cpu().numpy(), s_or) <= 1e-9, t
        f_gpu, _ = st.slice_loss(X, s_gpu)
        f_or, _ = slice_loss(data.X[t], orc.A, s_or, "poisson_log")
        assert abs(f_gpu - f_or) <= 1e-9 * abs(f_or), t
        sc_gpu = st.ktensor_score(s_gpu, B, T(data.S_true[t]))
        assert abs(sc_gpu - ktensor_score(orc.A, s_or, data.A_true, data.S_true[t])) <= 1e-9, t
        if t > POIS_H:
            A_now = [a.cpu().numpy() for a in st.factors()]
            ratio = deviance(data.X[t], A_now, s_gpu.cpu().numpy()) / deviance(data.X[t], data.A_true,
                                                                             data.S_true[t])
            assert 0.97 <= ratio <= 1.0 and sc_gpu >= 0.92, (t, ratio, sc_gpu)
    A_gpu = [a.cpu().numpy() for a in st.factors()]
    for k in range(3):
        assert rel_err(A_gpu[k], orc.A[k]) <= 1e-9
