"""FP64 oracle for the stratified sampled gradient (Section 4.3, Algorithm 6).

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

For a sparse slice with eta stored nonzeros out of omega = I1 I2 I3 entries
(zeta = omega - eta zeros), p nonzeros and q zeros are drawn uniformly with
replacement; zero candidates are drawn as uniform index tuples and rejected
when they hit a stored nonzero.  Each drawn entry contributes
    ytilde = (eta/p) df/dm(x, m)      for a nonzero draw,
    ytilde = (zeta/q) df/dm(0, m)     for a zero draw,
to the gradient tensor, and the factor and weight gradients are the MTTKRPs
of eqs. gcp_grad_A / gcp_grad_lambda with ytilde in place of y.  The window
slices are sampled the same way and weighted by w_h; the regularisation
gradients are exact.  The objective is estimated with the same draws and the
same weights applied to f.

The random draws are specified so that two independent implementations
produce the same samples: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011) with key (seed low 32 bits,
seed high 32 bits) and counter
    (sample number, slice time stamp, call number, stratum + 2 * attempt)
with stratum 0 for nonzeros and 1 for zeros.  A nonzero draw uses word 0:
index = floor(word0 * eta / 2^32).  A zero draw uses words 0..2:
i_k = floor(word_k * I_k / 2^32); attempt 0, 1, ... until the tuple is not a
stored nonzero (at most 64 attempts).
"""
from __future__ import annotations

import numpy as np

from .gcp import loss_dfdm, loss_f

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
MAX_ATTEMPTS = 64


def philox4x32_10(ctr, key):
    """ctr: (4, n) uint32-valued array, key: (k0, k1).  Returns (4, n)."""
    c = [np.asarray(ctr[i], dtype=np.uint64) & MASK32 for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return np.stack(c).astype(np.uint64)


def _scale(word, n):
    return ((np.asarray(word, np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def draw_nonzeros(seed: int, stamp: int, call: int, p: int, eta: int):
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    c = np.arange(p, dtype=np.uint64)
    ctr = [c, np.full(p, stamp & 0xFFFFFFFF, np.uint64), np.full(p, call & 0xFFFFFFFF, np.uint64),
           np.zeros(p, np.uint64)]
    return _scale(philox4x32_10(ctr, key)[0], eta)


def draw_zeros(seed: int, stamp: int, call: int, q: int, dims, nonzero_lin: np.ndarray):
    """Accepted zero coordinates (q x 3) and the attempt that produced each."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    c = np.arange(q, dtype=np.uint64)
    out = np.zeros((q, 3), np.int64)
    attempt_of = np.full(q, -1, np.int64)
    todo = np.arange(q)
    for a in range(MAX_ATTEMPTS):
        if todo.size == 0:
            break
        ctr = [c[todo], np.full(todo.size, stamp & 0xFFFFFFFF, np.uint64),
               np.full(todo.size, call & 0xFFFFFFFF, np.uint64),
               np.full(todo.size, 1 + 2 * a, np.uint64)]
        w = philox4x32_10(ctr, key)
        idx = np.stack([_scale(w[k], dims[k]) for k in range(3)], axis=1)
        lin = (idx[:, 0] * dims[1] + idx[:, 1]) * dims[2] + idx[:, 2]
        hit = np.isin(lin, nonzero_lin)
        ok = ~hit
        out[todo[ok]] = idx[ok]
        attempt_of[todo[ok]] = a
        todo = todo[hit]
    if todo.size:
        raise RuntimeError("zero sampling did not terminate")
    return out, attempt_of


def sampled_terms(loss, coo, s, A, seed, stamp, call, p, q):
    """Per-draw coordinates, x values and weights for one slice."""
    dims = coo.dims
    omega = int(np.prod(dims))
    eta = coo.coords.shape[0]
    zeta = omega - eta
    lin = (coo.coords[:, 0].astype(np.int64) * dims[1] + coo.coords[:, 1]) * dims[2] + coo.coords[:, 2]
    nz = draw_nonzeros(seed, stamp, call, p, eta) if p > 0 else np.zeros(0, np.int64)
    zc, _ = draw_zeros(seed, stamp, call, q, dims, lin) if q > 0 else (np.zeros((0, 3), np.int64), None)
    coords = np.concatenate([coo.coords[nz].astype(np.int64), zc], axis=0)
    x = np.concatenate([coo.vals[nz].astype(np.float64), np.zeros(q)])
    wgt = np.concatenate([np.full(p, eta / p if p else 0.0), np.full(q, zeta / q if q else 0.0)])
    return coords, x, wgt


def sampled_loss_grad(prob, call: int = 0):
    """(F~, G~^(1..3), g~_s) for a sparse problem (gcp_inputs.SparseProblem)."""
    A = [np.asarray(a, np.float64) for a in prob.A]
    R = A[0].shape[1]
    slices = [(prob.X_t, np.asarray(prob.s_t, np.float64), 1.0, prob.t)]
    for h, sl in enumerate(prob.X_hist):
        c = prob.w * prob.theta ** (prob.t - int(prob.t_hist[h]))
        slices.append((sl, np.asarray(prob.s_hist[h], np.float64), c, int(prob.t_hist[h])))
    G = [prob.lam * a.copy() for a in A]
    g_s = prob.mu * np.asarray(prob.s_t, np.float64).copy()
    F = 0.5 * prob.lam * sum(float(np.sum(a * a)) for a in A) + \
        0.5 * prob.mu * float(np.sum(np.asarray(prob.s_t, np.float64) ** 2))
    for n, (coo, s, c, stamp) in enumerate(slices):
        coords, x, wgt = sampled_terms(prob.loss, coo, s, A, prob.seed, stamp, call, prob.p, prob.q)
        rows = [A[k][coords[:, k]] for k in range(3)]
        m = np.sum(s[None, :] * rows[0] * rows[1] * rows[2], axis=1)
        F += c * float(np.sum(wgt * loss_f(prob.loss, x, m)))
        yt = c * wgt * loss_dfdm(prob.loss, x, m)
        for k in range(3):
            others = [rows[l] for l in range(3) if l != k]
            contrib = yt[:, None] * s[None, :] * others[0] * others[1]
            np.add.at(G[k], coords[:, k], contrib)
        if n == 0:
            g_s += np.sum(yt[:, None] * rows[0] * rows[1] * rows[2], axis=0)
    return F, G, g_s


# Call numbers of the objective estimates of Algorithm 5 within the factor
# and the weight solves of time step t: fixed for a whole solve (every epoch
# compares estimates over the same draws), different for the two solvers and
# for each slice, and apart from the gradient calls, which count up from 0.
def estimate_call(t: int) -> int:
    return 0x80000000 | (int(t) & 0x3FFFFFFF)


def weight_estimate_call(t: int) -> int:
    return 0xC0000000 | (int(t) & 0x3FFFFFFF)


def estimate_objective(prob, p_est: int, q_est: int, call: int) -> float:
    """Algorithm 5 for the factor solver: the sampled objective with p_est
    nonzero and q_est zero draws per slice, the exact regulariser of the
    factors and no weight regulariser (Algorithm 4 passes mu = 0)."""
    from types import SimpleNamespace
    est = SimpleNamespace(**vars(prob))
    est.p, est.q, est.mu = p_est, q_est, 0.0
    return sampled_loss_grad(est, call=call)[0]


def sampled_factor_epochs(prob, state, *, tau, kappa, tol=-np.inf, p_est, q_est, beta1=0.9, beta2=0.999, eps=1e-8,
                          lower=-np.inf, decay=0.1):
    """Algorithm 4 on a sparse problem: epochs of tau sampled-gradient ADAM
    steps (a new call number for every gradient), each judged by Algorithm
    5's estimate over draws fixed for the solve, with the ADAM Update of
    Algorithm 2 (roll-back, rate times decay, index back tau).  `state`
    holds A, u, v, the saved Ao, uo, vo, alpha, i and the next call number;
    it is updated in place.  Every scheduled step consumes a call number,
    also after the stopping test is met.  Returns the roll-back decisions."""
    from .adam import adam_step
    ecall = estimate_call(prob.t)
    call_end = state.call + tau * kappa
    prob.A = [a.copy() for a in state.A]
    F = estimate_objective(prob, p_est, q_est, ecall)
    rolled, state.F_hist, state.F_try = [], [F], []
    for _ in range(kappa):
        if not F > tol:
            break
        F_old = F
        for _ in range(tau):
            prob.A = state.A
            _, G, _ = sampled_loss_grad(prob, call=state.call)
            state.call += 1
            for k in range(3):
                state.A[k], state.u[k], state.v[k] = adam_step(state.A[k], G[k], state.u[k], state.v[k], state.i,
                                                               state.alpha, beta1, beta2, eps, lower)
            state.i += 1
        prob.A = state.A
        F = estimate_objective(prob, p_est, q_est, ecall)
        state.F_try.append(F)
        if F > F_old:
            state.A = [a.copy() for a in state.Ao]
            state.u = [a.copy() for a in state.uo]
            state.v = [a.copy() for a in state.vo]
            state.alpha *= decay
            state.i -= tau
            F = F_old
            rolled.append(True)
        else:
            state.Ao = [a.copy() for a in state.A]
            state.uo = [a.copy() for a in state.u]
            state.vo = [a.copy() for a in state.v]
            rolled.append(False)
        state.F_hist.append(F)
    state.F = F
    state.call = call_end
    return rolled


def sampled_temporal_sgd(prob, call: int, *, alpha, tau, kappa, tol=-np.inf, p_est, q_est, beta1=0.9, beta2=0.999,
                         eps=1e-8, lower=-np.inf, decay=0.1):
    """Algorithm 3 on a sparse slice X_t (prob.X_t, factors prob.A fixed):
    s <- 0, epochs of tau ADAM steps on sampled weight gradients of X_t
    alone (no history, no factor regulariser; a new call number per step,
    counting from `call`), each judged by Algorithm 5's estimate of
    sum f + mu/2 ||s||^2 over draws fixed for the solve.  Returns
    (s, info) with info.rolled, info.F (accepted estimates), info.F_try,
    info.alpha, info.iters and info.call (the next call number)."""
    from types import SimpleNamespace
    from .adam import adam_step
    R = np.asarray(prob.A[0]).shape[1]
    base = SimpleNamespace(**vars(prob))
    base.X_hist, base.s_hist, base.t_hist, base.lam = [], np.zeros((0, R)), np.zeros(0, np.int64), 0.0

    def estimate(s):
        e = SimpleNamespace(**vars(base))
        e.s_t, e.p, e.q = s, p_est, q_est
        return sampled_loss_grad(e, call=weight_estimate_call(prob.t))[0]

    s = np.zeros(R)
    u, v = np.zeros(R), np.zeros(R)
    so, uo, vo = s.copy(), u.copy(), v.copy()
    i, nxt, end = 0, call, call + tau * kappa
    F = estimate(s)
    info = SimpleNamespace(F=[F], F_try=[], rolled=[])
    for _ in range(kappa):
        if not F > tol:
            break
        F_old = F
        for _ in range(tau):
            g = SimpleNamespace(**vars(base))
            g.s_t = s
            gs = sampled_loss_grad(g, call=nxt)[2]
            nxt += 1
            s, u, v = adam_step(s, gs, u, v, i, alpha, beta1, beta2, eps, lower)
            i += 1
        F = estimate(s)
        info.F_try.append(F)
        if F > F_old:
            s, u, v = so.copy(), uo.copy(), vo.copy()
            alpha *= decay
            i -= tau
            F = F_old
            info.rolled.append(True)
        else:
            so, uo, vo = s.copy(), u.copy(), v.copy()
            info.rolled.append(False)
        info.F.append(F)
    info.alpha, info.iters, info.call = alpha, i, end
    return s, info
