#!/usr/bin/env python3
"""Benchmark of the streaming-GCP gradient step on one MI355X.

Default workload (the batched configuration): 64 independent streams whose
dense FP32 slices have dims drawn from U{50..300}^3, ranks from {8, 16, 32}
and windows from 4..16, Gaussian and Poisson-log losses mixed.  One step =
one gcp_batch_loss_grad: the objective and every gradient of all 64 streams
over their current slices and full windows, replayed as a captured HIP graph
with inputs resident in HBM.

Prints ONE JSON line: batched grad steps/s, ms per step (wall clock over K
replays), the median / p10 / p90 of per-replay HIP-event times, the unfused
("plain") path's time for the same 64 gradients on the same GPU, the
roofline entry (algorithmic bytes / median replay time), the error of the
GPU result against the FP64 oracle on a sample of streams, and the oracle's
rate on this host.  --workload selects the other legs (C2, C3, C5, ...),
each printing a line of its own.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sets", type=int, default=2,
                    help="independent C2 input sets (each its own stream and window) used in turn, "
                         "so that the data read per step is not served from the 256 MB last-level "
                         "cache")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--fused-only", action="store_true",
                    help="time the fused step only (for profiler runs)")
    ap.add_argument("--workload", default="c4", choices=["c2", "c3", "c3b", "c4", "c5", "c2m", "c2w", "c2step", "ops", "e5",
                                                      "e6", "e7"],
                    help="c4 (default) is the batched configuration the metric is quoted on; the others "
                         "print their own line")
    ap.add_argument("--kernel", default="auto", choices=["auto", "valu", "mfma"],
                    help="c2m: the dense data-term kernel (auto: chosen by the library)")
    ap.add_argument("--sampled-atomic", action="store_true",
                    help="c5: sum the MTTKRP rows with float atomics instead of the row-sorted lists")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="instead of the workload, run a plain device-to-device copy of this "
                         "many MiB a few times (calibrates the FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def copy_probe(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}), flush=True)
    return 0


# Sources of the C2 matrix-core kernel; the committed counter summary carries
# their sha256 and its traffic figure is used only while they are unchanged.
C2_KERNEL_SOURCES = ["paper_2110_14514_amd/csrc/mfma_tile.hpp",
                     "paper_2110_14514_amd/csrc/dense_mfma_poisson.hip",
                     "paper_2110_14514_amd/csrc/common.hpp"]


def _profiled_traffic(summary: str, sources):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated with a copy of known
    size), or None when the kernel sources differ from the ones profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().split()[0] if v.strip() else ""
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _time(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


# FP32 vector-ALU peak without packed FP32 instructions (which this build
# keeps out of every kernel): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz.
VALU_FP32_PEAK_TFLOPS = 78.6


def _roof(alg_bytes, alg_flops, kern_s, traffic=None, **extra):
    """Roofline entry of one kernel launch.  The binding roof is the one with
    the longer minimum time: algorithmic bytes at the HBM peak, or
    algorithmic FP32 flops at the FP32 matrix-core peak (the contraction's
    own dtype).  Both fractions are kept beside it."""
    gbs = alg_bytes / kern_s / 1e9
    tf = alg_flops / kern_s / 1e12
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = alg_flops / (FP32_PEAK_TFLOPS * 1e12)
    r = {"traffic": traffic, "kernel_ms": kern_s * 1e3, "alg_bytes_per_launch": alg_bytes,
         "alg_gflops_per_launch": alg_flops / 1e9,
         "roof_ms": {"hbm": t_hbm * 1e3, "fp32_mfma": t_mfma * 1e3},
         "hbm_GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
         "fp32_tflops": tf, "fp32_frac": tf / FP32_PEAK_TFLOPS}
    if t_mfma > t_hbm:
        r.update({"bound": "mfma", "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                  "frac": tf / FP32_PEAK_TFLOPS})
    else:
        r.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": gbs / HBM_PEAK_GBS})
    r.update(extra)
    return r


def _line(workload, value_unit, ms, steps, warmup, alg_bytes, alg_flops, kern_s, extra, bound="hbm"):
    ach = alg_bytes / kern_s / 1e9
    out = {"metric": "GCP grad steps/sec + achieved HBM GB/s (% peak), fused vs plain, err<=1e-5",
           "value": 1e3 / ms, "unit": value_unit, "n_gpus": 1, "ms_per_step": ms, "steps": steps,
           "warmup": warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": workload},
           "roofline": _roof(alg_bytes, alg_flops, kern_s)}
    if bound == "alu":
        tf = alg_flops / kern_s / 1e12
        out["roofline"].update({"bound": "alu", "achieved": tf, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": tf / VALU_FP32_PEAK_TFLOPS, "hbm_GBps": ach})
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_c3(args, bits=False):
    """C3: 1000x1000x64 binary slices, rank 32, window 20, Bernoulli-logit
    (bits: the same slices bit-packed, one bit per entry)."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream
    dims, R, H = (1000, 1000, 64), 32, 20
    print("bench: generating C3 on the device", file=sys.stderr, flush=True)
    X_t, A, s_t, Xh, Sh = gi.device_dense_window(dims, R, H, "bernoulli_logit", seed=2)
    if bits:
        X_t = gi.device_pack_bits(X_t)
        Xh = [gi.device_pack_bits(x) for x in Xh]
    st = Stream(dims, R, H, "bernoulli_logit", A, Xh, Sh, list(range(1, H + 1)),
                slice_kind="bits" if bits else "dense")
    del Xh
    torch.cuda.synchronize()
    out = (torch.empty(1, device="cuda"), [torch.empty(n, R, device="cuda") for n in dims],
           torch.empty(R, device="cuda"))
    fn = lambda: st.loss_grad(X_t, A, s_t, out=out)
    st.kernel_timing(True, args.steps)
    sec = _time(fn, args.steps, 0, torch.cuda.synchronize)
    ms, n = st.kernel_time()
    st.kernel_timing(False)
    assert st.sync() == 0
    omega = int(np.prod(dims))
    name = ("C3 bit-packed binary slices 1000x1000x64 (one bit per entry), rank 32, window 20, Bernoulli-logit"
            if bits else "C3 dense binary slices 1000x1000x64, rank 32, window 20, Bernoulli-logit")
    _line(name, "grad steps/s", sec * 1e3, args.steps, 0, (H + 1) * omega * (4 if not bits else 0.125),
          omega * (4 * R * (H + 1) + 8 * R), ms / max(n, 1) / 1e3, {})
    return 0


def _copy_ceiling(mib: int = 2048, reps: int = 5):
    """Measured HBM ceiling: GB/s (bytes read + written) of a device-to-device
    copy of `mib` MiB, the best of `reps` timed copies."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    return 2 * n * 4 / best / 1e9


def _gather_ceiling(A, ndraws: int, reps: int = 5):
    """Measured gather roof of the sampled path: draws/s of the library's
    gather probe (three random factor-row gathers and a 16-byte record per
    draw, nothing else) over the same factor matrices."""
    import ctypes
    import torch
    from paper_2110_14514_amd import _native as N
    lib = N.load()
    rec = torch.empty(ndraws * 4, device="cuda")
    st = torch.cuda.current_stream()
    args = [ctypes.c_void_p(a.data_ptr()) for a in A] + [a.shape[0] for a in A] + [A[0].shape[1], ndraws]
    call = lambda seed: N.check(lib.gcp_probe_gather(*args, seed, ctypes.c_void_p(rec.data_ptr()),
                                                     ctypes.c_void_p(st.cuda_stream)), "gcp_probe_gather")
    call(1)
    best = 1e30
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        call(2 + r)
        e1.record(st)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del rec
    return ndraws / best


def _cpu_info():
    """Host CPU model, NumPy's BLAS and the BLAS thread count (for the
    oracle's baseline line)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        dep = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        blas = f"{dep.get('name', '')} {dep.get('version', '')}".strip()
    except Exception:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    return model, blas, int(threads)


C4_KERNEL_SOURCES = ["paper_2110_14514_amd/csrc/mfma_tile.hpp", "paper_2110_14514_amd/csrc/dense_mfma.hip",
                     "paper_2110_14514_amd/csrc/dense_mfma_gaussian.hip",
                     "paper_2110_14514_amd/csrc/dense_mfma_poisson.hip", "paper_2110_14514_amd/csrc/common.hpp"]


def bench_c4(args):
    """C4: 64 streams, dims U{50..300}^3, rank {8,16,32}, window 4..16,
    Gaussian/Poisson-log; one step = one batched gcp_batch_loss_grad (all 64
    stream gradients), captured once as a HIP graph and replayed."""
    import torch
    import gcp_inputs as gi
    from oracle import gcp as og
    from paper_2110_14514_amd import Batch, Stream
    specs = gi.c4_specs()
    side = torch.cuda.Stream()       # graph capture needs a non-default stream
    torch.cuda.set_stream(side)
    plain = not (args.no_plain or args.fused_only)
    cpu_leg = not (args.no_cpu_baseline or args.fused_only)
    # oracle sample: per tile class (loss, rank tile, h-tiles, copy width) the
    # smallest stream, when its window holds at most 25M entries
    classes = {}
    for i, sp in enumerate(specs):
        key = (sp.loss, sp.rank > 16, sp.window + 1 > 16, sp.dims[2] % 4 == 0)
        es = int(np.prod(sp.dims)) * (sp.window + 1)
        if key not in classes or es < classes[key][0]:
            classes[key] = (es, i)
    sample = sorted(i for es, i in classes.values() if es <= 25_000_000) if cpu_leg else []
    streams, Xb, Sb, keep = [], [], [], {}
    tot_bytes = tot_flops = tot_es = 0
    print("bench: generating C4 on the device", file=sys.stderr, flush=True)
    for i, sp in enumerate(specs):
        X_t, A, s_t, Xh, Sh = gi.device_dense_window(sp.dims, sp.rank, sp.window, sp.loss, sp.seed)
        streams.append(Stream(sp.dims, sp.rank, sp.window, sp.loss, A, Xh, Sh,
                              list(range(1, sp.window + 1)), alpha_f=1e-4, tau_f=1, plain=plain))
        Xb.append(X_t)
        Sb.append(s_t)
        keep[i] = (A, Xh if i in sample else None, Sh)
        om, ns, R = int(np.prod(sp.dims)), sp.window + 1, sp.rank
        tot_es += om * ns
        tot_bytes += ns * om * 4 + 4 * R * sum(sp.dims) * 2 + 4 * R * (ns + 1)
        tot_flops += om * (4 * R * ns + 8 * R)
        del Xh
    torch.cuda.synchronize()
    b = Batch(streams, Xb, Sb)
    b.loss_grad()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=streams[0].hip_stream):
        b.loss_grad()
    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    K = max(args.steps, 1)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(side)
        g.replay()
        e1.record(side)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert b.sync_streams() == 0, "device reported a numeric failure"
    ms_per_step = (t1 - t0) * 1e3 / K
    rep = np.array(sorted(e0.elapsed_time(e1) for e0, e1 in ev))
    med, p10, p90 = (float(np.percentile(rep, q)) for q in (50, 10, 90))
    print(f"bench: batched step {ms_per_step:.3f} ms (replay median {med:.3f} ms)", file=sys.stderr, flush=True)

    # ---- unfused path: the same 64 gradients through the plain kernels ------
    plain_ms = None
    if plain:
        outs = [(torch.empty(1, device="cuda"), [torch.empty(n, sp.rank, device="cuda") for n in sp.dims],
                 torch.empty(sp.rank, device="cuda")) for sp in specs]

        def plain_step():
            for i, st in enumerate(streams):
                st.loss_grad(Xb[i], keep[i][0], Sb[i], plain=True, out=outs[i])
        plain_step()
        torch.cuda.synchronize()
        n_plain = 3
        c0 = time.perf_counter()
        for _ in range(n_plain):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - c0) * 1e3 / n_plain
        for st in streams:
            assert st.sync() == 0
        print(f"bench: plain {plain_ms:.3f} ms per 64 gradients", file=sys.stderr, flush=True)

    # ---- oracle: error of the GPU result and the CPU rate on the sample -----
    err, cpu = None, None
    if sample:
        host = lambda x: x.double().cpu().numpy()
        worst = {"loss": 0.0, "G_normwise": 0.0, "G_elementwise": 0.0, "g_s_normwise": 0.0,
                 "g_s_elementwise": 0.0}
        csec, ses = 0.0, 0
        from types import SimpleNamespace
        for i in sample:
            sp = specs[i]
            A, Xh, Sh = keep[i]
            prob = SimpleNamespace(X_t=host(Xb[i]), A=[host(a) for a in A], s_t=host(Sb[i]),
                                   X_hist=[host(x) for x in Xh], s_hist=host(Sh), t_hist=np.arange(1, sp.window + 1),
                                   t=sp.window + 1, w=1.0, theta=1.0, lam=0.0, mu=0.0, loss=sp.loss)
            c0 = time.perf_counter()
            F = og.objective(prob)
            Gr, gsr = og.gradient(prob)
            csec += time.perf_counter() - c0
            ses += int(np.prod(sp.dims)) * (sp.window + 1)
            loss, G, g_s = b.outputs[i]
            scale = og.loss_terms_abs(prob)
            worst["loss"] = max(worst["loss"], abs(float(loss.item()) - F) / max(abs(F), scale))
            for k in range(3):
                gk = host(G[k])
                worst["G_normwise"] = max(worst["G_normwise"], float(np.linalg.norm(gk - Gr[k]) / np.linalg.norm(Gr[k])))
                colmax = np.maximum(np.max(np.abs(Gr[k]), axis=0), np.sqrt(np.mean(Gr[k] * Gr[k])))
                worst["G_elementwise"] = max(worst["G_elementwise"],
                                             float(np.max(np.abs(gk - Gr[k]) / np.where(colmax > 0, colmax, 1.0))))
            gv = host(g_s)
            worst["g_s_normwise"] = max(worst["g_s_normwise"], float(np.linalg.norm(gv - gsr) / np.linalg.norm(gsr)))
            worst["g_s_elementwise"] = max(worst["g_s_elementwise"], float(np.max(np.abs(gv - gsr)) / np.max(np.abs(gsr))))
        err = dict(worst, streams_checked=sample)
        model, blas, threads = _cpu_info()
        share = ses / tot_es
        cpu = {"value": share / csec, "unit": "batched grad steps/s (64 streams each)", "cores": threads,
               "kind": "oracle", "cpu_model": model, "blas": blas, "numpy": np.__version__,
               "sample": f"FP64 NumPy oracle objective+gradient of {len(sample)} of the 64 streams (the smallest of "
                         f"each tile class up to 25M window entries: streams {sample}), {csec:.1f} s for "
                         f"{100 * share:.1f}% of the step's entry-slices, scaled to one batched step"}
    traffic = _profiled_traffic("batch_c4.txt", C4_KERNEL_SOURCES)
    ach = tot_bytes / (med / 1e3) / 1e9
    copy_gbs = _copy_ceiling()
    res = {
        "metric": "GCP grad steps/sec + achieved HBM GB/s (% peak), fused vs plain, err<=1e-5",
        "value": 1e3 / ms_per_step, "unit": "batched grad steps/s (64 streams each)", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C4: 64 independent streams, dense FP32 slices with dims U{50..300}^3, rank "
                               "{8,16,32}, window 4..16, Gaussian/Poisson-log mixed; one gcp_batch_loss_grad "
                               "(objective and all gradients of the 64 streams) replayed as a HIP graph",
                   "streams": len(specs), "entry_slices_per_step": tot_es, "parallelism": "single GPU"},
        "replay_ms": {"median": med, "p10": p10, "p90": p90, "replays": K},
        "stream_steps_per_s": len(specs) * 1e3 / ms_per_step,
        "roofline": _roof(tot_bytes, tot_flops, med / 1e3, traffic,
                          kernel="batched gradient step (tile kernels and their fixed-order reduce, one graph)",
                          measured_copy_GBps=copy_gbs, hbm_frac_of_measured_copy=ach / copy_gbs),
        "plain_ms_per_step": plain_ms,
        "fused_vs_plain": (plain_ms / ms_per_step) if plain_ms else None,
        "err_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_c2m(args):
    """C2 shape with the model-difference history (eq. gcp_stream_problem_2):
    the window keeps the 10 weights only; a step reads X_t once and adds the
    history term through R x R Gram matrices."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream
    dims, R, H, loss = (200, 200, 200), 16, 10, "poisson_log"
    prob = gi.c2_problem(seed=1, dims=dims, rank=R, window=H)
    g = np.random.default_rng(5)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    A_old = [a + 0.05 * g.uniform(-1, 1, size=a.shape) for a in prob.A]
    st = Stream(dims, R, H, loss, [T(a) for a in A_old], [], T(prob.s_hist), list(prob.t_hist),
                hist="model", kernel=args.kernel)
    X_t, A, s_t = T(prob.X_t), [T(a) for a in prob.A], T(prob.s_t)
    out = (torch.empty(1, device="cuda"), [torch.empty(n, R, device="cuda") for n in dims],
           torch.empty(R, device="cuda"))
    fn = lambda: st.loss_grad(X_t, A, s_t, out=out)
    for _ in range(args.warmup):
        fn()
    st.kernel_timing(True, args.steps)
    sec = _time(fn, args.steps, 0, torch.cuda.synchronize)
    ms, n = st.kernel_time()
    st.kernel_timing(False)
    assert st.sync() == 0
    omega = int(np.prod(dims))
    _line("C2 shape with the model-difference history: 200x200x200 Poisson-count slice, rank 16, "
          "window of 10 weights, Poisson-log", "grad steps/s", sec * 1e3, args.steps, args.warmup,
          omega * 4, omega * (4 * R + 8 * R), ms / max(n, 1) / 1e3, {})
    return 0


def bench_c2w(args):
    """C2 shape, temporal-weight solve of Algorithm 3 on the device (Poisson
    counts around a planted rank-16 log-rate model, factors fixed): ADAM
    epochs on s_t with the factors fixed, tau_w = 100 steps per epoch and
    kappa_w = 20 epochs (the paper's experiment settings), so one solve is
    20 x 101 + 1 passes over X_t.  Rate: solves per second; the roofline
    entry is per pass (whole solve time over its passes, gaps included)."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream
    dims, R, loss = (200, 200, 200), 16, "poisson_log"
    tau, kappa = 100, 20
    X, A, _ = gi.weight_problem(dims, R, loss, 1)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    st = Stream(dims, R, 0, loss, [T(a) for a in A], tsolve="sgd", tau_w=tau, kappa_w=kappa, alpha_w=0.05)
    X_t = T(X)
    s = torch.empty(R, device="cuda")
    fn = lambda: st.solve_st(X_t, out=s)
    cs = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    ev0.record(cs)
    sec = _time(fn, args.steps, 0, torch.cuda.synchronize)
    ev1.record(cs)
    torch.cuda.synchronize()
    assert st.sync() == 0
    info = st.solve_info()
    passes = kappa * (tau + 1) + 1
    per_pass = ev0.elapsed_time(ev1) / 1e3 / args.steps / passes
    omega = int(np.prod(dims))
    _line("C2 shape temporal-weight solve (Algorithm 3): 200x200x200 Poisson-count slice, rank 16, "
          "100 ADAM steps x 20 epochs", "weight solves/s", sec * 1e3, args.steps, args.warmup,
          omega * 4, omega * (4 * R + 8), per_pass,
          {"passes_per_solve": passes, "solve_F": info["F"], "rolled_epochs": sum(info["rolled"])}, bound="alu")
    return 0


def bench_c2step(args):
    """Whole OnlineGCP time steps (Algorithm 1) at the C2 shape with both SGD
    solvers on the device: Algorithm 3 for s_t (tau_w = 100, kappa_w = 20,
    alpha_w = 1) and Algorithm 4's epochs for the factors (tau_f = 100,
    kappa_f = 10, alpha_f = 1e-4), the iteration counts and rates of the
    paper's synthetic Poisson experiment, over a window of 10 stored slices.
    Each step takes a new slice; rate: time steps per second."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream
    dims, R, H, loss = (200, 200, 200), 16, 10, "poisson_log"
    X_t, A, s_t, Xh, Sh = gi.device_dense_window(dims, R, H, loss, seed=1)
    st = Stream(dims, R, H, loss, A, Xh, Sh, list(range(1, H + 1)), tsolve="sgd", tau_w=100, kappa_w=20,
                alpha_w=1.0, tau_f=100, kappa_f=10, alpha_f=1e-4, kernel=args.kernel)
    del Xh
    new = [gi.device_dense_window(dims, R, 0, loss, seed=100 + k)[0] for k in range(2)]
    torch.cuda.synchronize()
    k = [0]

    def fn():
        st.step(new[k[0] % 2])
        k[0] += 1

    steps = max(1, min(args.steps, 5))
    warm = max(1, min(args.warmup, 1))
    sec = _time(fn, steps, warm, torch.cuda.synchronize)
    assert st.sync() == 0
    fi, wi = st.factor_info(), st.solve_info()
    omega = int(np.prod(dims))
    passes = (100 + 1) * 10 + 1
    out = {"metric": "OnlineGCP time steps/sec (both SGD solvers on the device)", "value": 1.0 / sec,
           "unit": "time steps/s", "n_gpus": 1, "ms_per_step": sec * 1e3, "steps": steps, "warmup": warm,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "C2 shape OnlineGCP steps: 200x200x200 Poisson-count slices, rank 16, window "
                                  "10, tau 100, kappa_w 20, kappa_f 10"},
           "fused_passes_per_step": passes, "weight_passes_per_step": 20 * 101 + 1,
           "alg_bytes_per_fused_pass": 4 * (H + 1) * omega,
           "last_factor_epochs": fi["epochs"], "last_factor_rollbacks": sum(fi["rolled"]),
           "last_weight_rollbacks": sum(wi["rolled"])}
    print(json.dumps(out), flush=True)
    return 0


def bench_ops(args):
    """The other calls of a time step at the C2 shape (200^3, rank 16,
    window 10), each timed with HIP events on the stream the library uses:
    the least-squares temporal solve (one pass over X_t plus an R x R FP64
    solve), a gradient-only Gaussian call with and without the identity
    path (Section 5: no model evaluation), the loss and gradient under the
    paper's two identity-link losses (Poisson identity, Bernoulli odds), one
    factor update (gradient, ADAM step, A_old copy and the
    window push of a 32 MB slice), and the differentiation wrapper's forward
    + backward (two fused passes).  Algorithmic bytes: 4 B per entry of X_t
    for the solve; the gradient's 352 MB plus the 32 MB slice push for the
    update; twice the gradient's bytes for forward + backward."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream, gcp_loss
    dims, R, H = (200, 200, 200), 16, 10
    omega = int(np.prod(dims))
    X_t, A, s_t, Xh, Sh = gi.device_dense_window(dims, R, H, "poisson_log", seed=1)
    cs = torch.cuda.current_stream()

    def timed(fn, n):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cs)
        for _ in range(n):
            fn()
        e1.record(cs)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e-3

    n = max(5, min(args.steps, 50))
    g = Stream(dims, R, H, "gaussian", A, Xh, Sh, list(range(1, H + 1)))
    t_ls = timed(lambda: g.solve_st(X_t), n)
    # the LS weights' error against the oracle's FP64 solve (explicit Z):
    # the FP32 stream, and an FP64 stream over the same values
    from oracle.solve import ls_temporal
    s32 = g.solve_st(X_t).double().cpu().numpy()
    A64 = [a.double() for a in A]
    g64 = Stream(dims, R, 0, "gaussian", A64)
    s64 = g64.solve_st(X_t.double()).cpu().numpy()
    assert g64.sync() == 0
    del g64
    s_ref = ls_temporal(X_t.double().cpu().numpy(), [a.cpu().numpy() for a in A64])
    ls_err = lambda v: float(np.linalg.norm(v - s_ref) / np.linalg.norm(s_ref))
    t_gg = timed(lambda: g.loss_grad(X_t, A, s_t, want_loss=False), n)
    del g
    gi_ = Stream(dims, R, H, "gaussian", A, Xh, Sh, list(range(1, H + 1)), gauss_identity=True)
    t_gi = timed(lambda: gi_.loss_grad(X_t, A, s_t, want_loss=False), n)
    del gi_
    # The paper's identity-link losses need a nonnegative model: the same
    # factors in absolute value, the count data as is, its support as 0/1 data.
    Ap = [a.abs().contiguous() for a in A]
    q = Stream(dims, R, H, "poisson_id", Ap, Xh, Sh, list(range(1, H + 1)))
    t_pid = timed(lambda: q.loss_grad(X_t, Ap, s_t), n)
    assert q.sync() == 0
    del q
    Xb, Xhb = (X_t > 0).float(), [(x > 0).float() for x in Xh]
    q = Stream(dims, R, H, "bernoulli_odds", Ap, Xhb, Sh, list(range(1, H + 1)))
    t_bod = timed(lambda: q.loss_grad(Xb, Ap, s_t), n)
    assert q.sync() == 0
    del q, Xb, Xhb
    p = Stream(dims, R, H, "poisson_log", A, Xh, Sh, list(range(1, H + 1)), tau_f=1, alpha_f=1e-4)
    t_grad = timed(lambda: p.loss_grad(X_t, A, s_t), n)
    t_upd = timed(lambda: p.update_factors(X_t, s_t), n)
    Al = [a.clone().requires_grad_(True) for a in A]
    sl = s_t.clone().requires_grad_(True)

    def fwd_bwd():
        F = gcp_loss(p, X_t, Al, sl)
        F.backward()

    t_ad = timed(fwd_bwd, n)
    assert p.sync() == 0
    grad_bytes = 4 * (H + 1) * omega
    out = {"metric": "time-step calls at the C2 shape", "value": 1.0 / t_upd, "unit": "factor updates/s",
           "n_gpus": 1, "steps": n, "warmup": 2, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "C2 shape 200x200x200, rank 16, window 10: LS solve (Gaussian), factor update "
                                  "and autograd forward+backward (Poisson-log)"},
           "ls_solve_ms": t_ls * 1e3, "ls_solve_GBps": 4 * omega / t_ls / 1e9,
           "ls_rel_err_vs_oracle": {"fp32_stream": ls_err(s32), "fp64_stream": ls_err(s64)},
           "gaussian_grad_only_ms": t_gg * 1e3, "gaussian_grad_identity_ms": t_gi * 1e3,
           "grad_ms": t_grad * 1e3, "grad_poisson_identity_ms": t_pid * 1e3,
           "grad_bernoulli_odds_ms": t_bod * 1e3,
           "update_factors_ms": t_upd * 1e3, "update_GBps": (grad_bytes + 8 * omega) / t_upd / 1e9,
           "update_minus_grad_ms": (t_upd - t_grad) * 1e3,
           "autograd_fwd_bwd_ms": t_ad * 1e3, "autograd_GBps": 2 * grad_bytes / t_ad / 1e9}
    print(json.dumps(out), flush=True)
    return 0


def bench_e5(args):
    """Matrix slices at the shape of the paper's synthetic Gaussian experiment:
    300 x 300 slices, rank 20, window 50 (Table of hyperparameters); one
    gradient over X_t and the 50 stored slices, with each dense kernel."""
    import torch
    from paper_2110_14514_amd import Stream
    dims, R, H = (300, 300), 20, 50
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    Xs = [torch.randn(dims, generator=g, device="cuda") for _ in range(H + 1)]
    A = [(torch.rand(n, R, generator=g, device="cuda") - 0.5).contiguous() for n in dims]
    S = torch.rand(H + 1, R, generator=g, device="cuda") + 0.5
    res = {}
    for kernel in ("valu", "mfma", "auto"):
        st = Stream(dims, R, H, "gaussian", A, Xs[1:], S[1:].contiguous(), list(range(1, H + 1)), kernel=kernel)
        out = (torch.empty(1, device="cuda"), [torch.empty(n, R, device="cuda") for n in dims],
               torch.empty(R, device="cuda"))
        fn = lambda: st.loss_grad(Xs[0], A, S[0], out=out)
        for _ in range(args.warmup):
            fn()
        st.kernel_timing(True, args.steps)
        sec = _time(fn, args.steps, 0, torch.cuda.synchronize)
        ms, n = st.kernel_time()
        st.kernel_timing(False)
        assert st.sync() == 0
        res[kernel] = (sec, ms / max(n, 1) / 1e3)
        del st
    sec, ks = res["auto"]
    omega = 300 * 300
    _line("E5 shape: 300x300 Gaussian matrix slices, rank 20, window 50", "grad steps/s", sec * 1e3, args.steps,
          args.warmup, 4 * (H + 1) * omega, omega * (H + 1) * 4 * R, ks,
          {"valu_kernel_ms": res["valu"][1] * 1e3, "mfma_kernel_ms": res["mfma"][1] * 1e3})
    return 0


def bench_c5(args):
    """C5: sampled-sparse path, 2000x2000x500 COO slices (2M nonzeros),
    rank 32, window 8, p = q = 2M draws per slice, Poisson-log.  With
    ``--workload e6`` / ``e7`` the same call at the paper's count-data shape:
    263x263x24 slices at 3.8% density, rank 50, window 30, 10k + 10k (e6) or
    50k + 50k (e7) draws per slice."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream
    print("bench: generating", args.workload, file=sys.stderr, flush=True)
    if args.workload == "c5":
        prob = gi.sparse_problem()
        label = "C5 sampled COO slices 2000x2000x500, 2M nonzeros, rank 32, window 8, p=q=2M, Poisson-log"
    else:
        pq = 10000 if args.workload == "e6" else 50000
        prob = gi.sparse_problem(dims=(263, 263, 24), rank=50, window=30, nnz=63000, p=pq, q=pq, seed=6,
                                 loss="poisson_log")
        label = f"sampled COO slices 263x263x24 at 3.8%, rank 50, window 30, p=q={pq}, Poisson-log"
    T = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    coo = lambda sl: (T(sl.coords, torch.int32), T(sl.vals))
    R, H = prob.rank, len(prob.X_hist)
    st = Stream(prob.dims, R, H, prob.loss, [T(a) for a in prob.A], [coo(x) for x in prob.X_hist],
                T(prob.s_hist), list(prob.t_hist), seed=prob.seed, slice_kind="coo",
                max_nnz=prob.X_t.coords.shape[0], p=prob.p, q=prob.q,
                sampled_atomic=args.sampled_atomic)
    Xt = coo(prob.X_t)
    A = [T(a) for a in prob.A]
    s_t = T(prob.s_t)
    out = (torch.empty(1, device="cuda"), [torch.empty(n, R, device="cuda") for n in prob.dims],
           torch.empty(R, device="cuda"))
    fn = lambda: st.loss_grad(Xt, A, s_t, out=out)
    for _ in range(args.warmup):
        fn()
    st.kernel_timing(True, args.steps)
    sec = _time(fn, args.steps, 0, torch.cuda.synchronize)
    ms, n = st.kernel_time()
    st.kernel_timing(False)
    assert st.sync() == 0
    draws = (H + 1) * (prob.p + prob.q)
    # algorithmic bytes: a nonzero draw reads its coordinates and value (16 B);
    # a zero draw is a generated tuple plus one membership probe (8 B)
    alg = (H + 1) * (prob.p * 16 + prob.q * 8)
    kern_s = ms / max(n, 1) / 1e3
    # gather roof: the draw kernel gathers three factor rows per draw and the
    # row-sorted reduction two per record, three records per draw (nine rows
    # per draw; the float-atomic variant: three); the probe measures draws/s
    # at three rows per draw on the same factors
    probe = _gather_ceiling(A, draws)
    rows_per_draw = 3 if args.sampled_atomic else 9
    gath = draws * rows_per_draw / kern_s
    roof = 3 * probe
    _line(label, "grad steps/s", sec * 1e3, args.steps, args.warmup, alg,
          draws * 16 * R, kern_s,
          {"draws_per_step": draws, "draws_per_s": draws / kern_s,
           "reduction": "atomic" if args.sampled_atomic else "row-sorted",
           "gather_roof": {"bound": "gather", "achieved": gath, "peak": roof, "unit": "factor rows/s",
                           "frac": gath / roof, "rows_per_draw": rows_per_draw,
                           "probe_draws_per_s": probe}})
    return 0


def bench_c2(args):
    """C2: dense Poisson-count slices of 200x200x200 FP32, rank 16, window 10,
    Poisson-log; one gcp_loss_grad over X_t and 10 stored slices, two input
    sets in turn (704 MB, beyond the 256 MB last-level cache)."""
    import torch
    import gcp_inputs as gi
    from paper_2110_14514_amd import Stream

    dims, R, H, loss = (200, 200, 200), 16, 10, "poisson_log"
    nsets = max(1, args.sets)
    print(f"bench: generating workload {dims} R={R} H={H} {loss}, {nsets} input set(s)",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    plain = not (args.no_plain or args.fused_only)
    sets = []
    for k in range(nsets):
        pk = gi.c2_problem(seed=1 + 1000 * k, dims=dims, rank=R, window=H)
        Xh = [T(x) for x in pk.X_hist]
        A = [T(a) for a in pk.A]
        stk = Stream(dims, R, H, loss, A, Xh, T(pk.s_hist), list(pk.t_hist), plain=plain and k == 0)
        del Xh
        sets.append({"prob": pk, "st": stk, "X_t": T(pk.X_t), "A": A, "s_t": T(pk.s_t)})
    prob, st = sets[0]["prob"], sets[0]["st"]
    torch.cuda.synchronize()
    out = (torch.empty(1, device=dev), [torch.empty(n, R, device=dev) for n in dims],
           torch.empty(R, device=dev))

    def run(n, plain_path=False):
        for i in range(n):
            sk = sets[0] if plain_path else sets[i % nsets]
            sk["st"].loss_grad(sk["X_t"], sk["A"], sk["s_t"], plain=plain_path, out=out)

    # ---- fused path -------------------------------------------------------
    print("bench: warmup", file=sys.stderr, flush=True)
    run(args.warmup)
    torch.cuda.synchronize()
    for sk in sets:
        sk["st"].kernel_timing(True, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = 0.0, 0
    for sk in sets:
        m_, n_ = sk["st"].kernel_time()
        sk["st"].kernel_timing(False)
        kern_ms += m_
        kern_n += n_
        assert sk["st"].sync() == 0, "device reported a numeric failure"
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print(f"bench: fused {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)
    run(1)          # one more call on set 0: the result compared with the oracle
    torch.cuda.synchronize()
    gpu_res = (float(out[0].item()), [g.double().cpu().numpy() for g in out[1]],
               out[2].double().cpu().numpy())

    ns = H + 1
    omega = int(np.prod(dims))
    alg_bytes = ns * omega * 4 + 4 * R * sum(dims) * 2 + 4 * R * (ns + 1)
    alg_flops = omega * (4 * R * ns + 8 * R)
    kavg_s = kern_ms / max(kern_n, 1) / 1e3
    achieved = alg_bytes / kavg_s / 1e9

    # ---- plain path -------------------------------------------------------
    plain_ms = None
    if plain:
        run(2, True)
        torch.cuda.synchronize()
        n_plain = max(3, args.steps // 10)
        t0 = time.perf_counter()
        run(n_plain, True)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / n_plain
        assert st.sync() == 0
        print(f"bench: plain {plain_ms:.4f} ms/step", file=sys.stderr, flush=True)

    # ---- CPU oracle ---------------------------------------------------------
    cpu = None
    err = None
    if not (args.no_cpu_baseline or args.fused_only):
        from oracle import gcp as og
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        p64 = prob.promoted()
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        F = og.objective(p64)
        G, gs = og.gradient(p64)
        csec = time.perf_counter() - c0
        scale = og.loss_terms_abs(p64)
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        err = {"loss": abs(gpu_res[0] - F) / max(abs(F), scale),
               **{f"G{k + 1}": rel(gpu_res[1][k], G[k]) for k in range(3)},
               "g_s": rel(gpu_res[2], gs)}
        cpu = {"value": 1.0 / csec, "unit": "grad steps/s", "cores": int(cores),
               "kind": "oracle",
               "sample": "one full objective+gradient evaluation of the same 200^3 x 11-slice "
                         "workload (FP64 NumPy oracle, BLAS threads as listed)"}

    traffic = _profiled_traffic("fused_dense_c2.txt", C2_KERNEL_SOURCES)
    res = {
        "metric": "GCP grad steps/sec + achieved HBM GB/s (% peak), fused vs plain, err<=1e-5",
        "value": 1e3 / ms_per_step,
        "unit": "grad steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2 dense Poisson-count slices 200x200x200, rank 16, window 10, "
                               "Poisson-log loss, one gcp_loss_grad over X_t and 10 stored slices",
                   "dims": list(dims), "rank": R, "window": H, "loss": loss,
                   "input_sets": nsets, "parallelism": "single GPU"},
        "roofline": _roof(alg_bytes, alg_flops, kavg_s, traffic, kernel="fused dense objective+gradient kernel"),
        "plain_ms_per_step": plain_ms,
        "fused_vs_plain": (plain_ms / ms_per_step) if plain_ms else None,
        "err_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    return {"c2": bench_c2, "c3": bench_c3, "c3b": lambda a: bench_c3(a, bits=True), "c4": bench_c4, "c5": bench_c5, "c2m": bench_c2m, "c2w": bench_c2w,
            "c2step": bench_c2step, "ops": bench_ops, "e5": bench_e5, "e6": bench_c5,
            "e7": bench_c5}[args.workload](args)

if __name__ == "__main__":
    sys.exit(main())
