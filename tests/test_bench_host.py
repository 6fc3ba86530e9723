"""Host-side checks of bench.py's bookkeeping: the binding-roof choice, the
gate that ties a committed counter summary to the kernel sources it was
taken on, and the one-GPU guard.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_roof_picks_hbm_when_bytes_take_longer():
    # 8 GB at 8 TB/s = 1 ms; 1 GFLOP at 157.3 TFLOP/s is far shorter
    r = bench._roof(8e9, 1e9, 2e-3)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["roof_ms"]["hbm"] == pytest.approx(1.0)
    assert r["fp32_frac"] == pytest.approx(1e9 / 2e-3 / 1e12 / bench.FP32_PEAK_TFLOPS)


def test_roof_picks_mfma_when_flops_take_longer():
    # 314.6 GFLOP at 157.3 TFLOP/s = 2 ms; 1 GB at 8 TB/s = 0.125 ms
    r = bench._roof(1e9, 314.6e9, 4e-3, traffic=1.5e9, kernel="k")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == bench.FP32_PEAK_TFLOPS
    assert r["frac"] == pytest.approx(0.5)
    assert r["hbm_frac"] == pytest.approx(1e9 / 4e-3 / 1e9 / bench.HBM_PEAK_GBS)
    assert r["traffic"] == 1.5e9 and r["kernel"] == "k"


@pytest.mark.parametrize("summary,sources", [("batch_c4.txt", bench.C4_KERNEL_SOURCES),
                                             ("fused_dense_c2.txt", bench.C2_KERNEL_SOURCES)])
def test_committed_counter_summaries_match_the_sources(summary, sources):
    """The HBM traffic a bench line reports comes from a committed counter
    summary; it must have been taken on the kernel sources as they stand."""
    t = bench._profiled_traffic(summary, sources)
    assert t is not None, f"profiles/{summary} was taken on other kernel sources"
    assert t > 0


def test_traffic_gate_rejects_other_sources():
    assert bench._profiled_traffic("fused_dense_c2.txt", bench.C2_KERNEL_SOURCES[:1]) is None
    assert bench._profiled_traffic("no_such_summary.txt", bench.C2_KERNEL_SOURCES) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
