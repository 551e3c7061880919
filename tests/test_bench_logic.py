"""Host logic of bench.py that feeds the reported line: the roofline entries'
arithmetic, the traffic figures' validity check against the kernel sources,
and the refusal of more than one GPU (one GPU's throughput is the value)."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _row(precision="fp32", kc=160, pairs=812_462, ms=1.65):
    return {"plan": {"m2l_rank": kc, "v_pairs": pairs, "p2p_pairs": 8_214_871_086}, "m2l_gemm_ms": ms,
            "precision": precision, "p2p_ms": 4.12}


def test_m2l_roofline_fp32():
    r = bench.m2l_roofline(_row(), learned_fp32=True)
    flops = 2.0 * 160 * 160 * 4 * 812_462
    assert r["flops_per_launch"] == flops
    assert r["achieved"] == pytest.approx(flops / 1.65e-3 / 1e12)
    assert r["peak"] == 157.3 and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["kernel"] == "gemm_f32_strip<5>"


def test_m2l_roofline_split_bf16_counts_three_passes():
    r = bench.m2l_roofline(_row("split_bf16", kc=224, ms=1.0))
    assert r["flops_per_launch"] == 3 * 2.0 * 224 * 224 * 4 * 812_462
    assert r["peak"] == 2500.0 and r["kernel"] == "gemm_bf16x3_mfma"
    assert r["traffic"] is None                # counters cover the learned FP32 launch only


def test_m2l_roofline_absent_without_compression():
    assert bench.m2l_roofline(_row(kc=0)) is None
    assert bench.m2l_roofline(_row(ms=0.0)) is None


def test_p2p_roofline():
    r = bench.p2p_roofline("Stokeslet", _row())
    assert r["achieved"] == pytest.approx(28 * 8_214_871_086 / 4.12e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3) and r["bound"] == "alu"


def test_traffic_is_reported_only_for_matching_sources(tmp_path, monkeypatch):
    # a summary gives its figure (or None once the kernel sources moved on:
    # a reported figure must never describe other code)
    for prof in (bench.PROFILE, bench.PROFILE_M2L):
        t = bench.measured_traffic(prof)
        assert t is None or t > 1e9
    # a changed source hides the figure
    src = tmp_path / "kernels.hip"
    src.write_bytes(open(bench.KERNEL_SOURCES[0], "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)] + bench.KERNEL_SOURCES[1:])
    assert bench.measured_traffic() is None and bench.measured_traffic(bench.PROFILE_M2L) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""
