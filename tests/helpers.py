"""Shared test helpers: move a synthetic problem to the device, run the HIP
path through the C ABI, and compare with the oracle normwise and per element
(each element against its column's largest reference value)."""
from __future__ import annotations

import numpy as np

TOL = 1e-5   # normwise relative tolerance for FP32 results against FP64


def rel_err(got, ref) -> float:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def elem_err(got, ref) -> float:
    """Largest per-element error, each element against the larger of the
    largest |value| of its column of the reference (a vector is one column)
    and the reference's RMS value: a wrong short row or a wrong rank column
    shows here even when the matrix norm hides it, while a column of a single
    entry (a mode of size 1) is not held to the relative error of one
    cancelling FP32 sum."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if not ref.size:
        return 0.0
    if ref.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    scale = np.maximum(np.max(np.abs(ref), axis=0), np.sqrt(np.mean(ref * ref)))
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(got - ref) / scale[None, :]))


def grad_err(got, ref) -> float:
    """max(normwise, per-element) error of a gradient against the oracle's."""
    return max(rel_err(got, ref), elem_err(got, ref))


def loss_err(got: float, ref: float, scale: float) -> float:
    """|F - F*| / max(|F*|, sum |terms|): the objective can cross zero."""
    return abs(float(got) - float(ref)) / max(abs(float(ref)), float(scale), 1e-300)


def to_device(prob, device="cuda"):
    import torch
    dt = torch.float64 if prob.dtype == np.float64 else torch.float32
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    return {
        "X_t": T(prob.X_t),
        "A": [T(a) for a in prob.A],
        "s_t": T(prob.s_t),
        "X_hist": [T(x) for x in prob.X_hist],
        "s_hist": T(np.asarray(prob.s_hist).reshape(len(prob.X_hist), prob.rank))
        if len(prob.X_hist) else None,
        "t_hist": [int(v) for v in prob.t_hist],
    }


def make_stream(prob, dev, plain=False, **kw):
    from paper_2110_14514_amd import Stream
    return Stream(prob.dims, prob.rank, len(prob.X_hist), prob.loss, dev["A"],
                  dev["X_hist"], dev["s_hist"], dev["t_hist"], w=prob.w, theta=prob.theta,
                  lam=prob.lam, mu=prob.mu, plain=plain, **kw)


def gpu_loss_grad(prob, plain=False, stream=None, kernel="auto"):
    import torch
    dev = to_device(prob)
    st = stream or make_stream(prob, dev, plain=plain, kernel=kernel)
    loss, G, g_s = st.loss_grad(dev["X_t"], dev["A"], dev["s_t"], plain=plain)
    torch.cuda.synchronize()
    code = st.sync()
    out = (float(loss.item()), [g.double().cpu().numpy() for g in G], g_s.double().cpu().numpy())
    return out, code, st


def compare(prob, got, oracle_mod):
    p64 = prob.promoted()
    F = oracle_mod.objective(p64)
    G, gs = oracle_mod.gradient(p64)
    scale = oracle_mod.loss_terms_abs(p64)
    errs = {"loss": loss_err(got[0], F, scale)}
    for k in range(3):
        errs[f"G{k + 1}"] = rel_err(got[1][k], G[k])
        errs[f"G{k + 1}_elem"] = elem_err(got[1][k], G[k])
    errs["g_s"] = rel_err(got[2], gs)
    errs["g_s_elem"] = elem_err(got[2], gs)
    return errs
