"""Host logic of bench.py: the per-step bytes model, the launch count of
blocked runs, the roofline it reports (HBM while the per-step model bounds the
kernel, the ALU roofline past it), the rule that counter traffic is reported
only for the kernel sources it was measured on, and the refusal of more than
one GPU.  No device is used."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADLINE = SimpleNamespace(name="quaternary_3d_d3q7_512x512x512", lattice="D3Q7", N=4, nodes=512 ** 3,
                           precision="f32")
TERNARY_2D = SimpleNamespace(name="ternary_2d_d2q5_4096x4096", lattice="D2Q5", N=3, nodes=4096 ** 2,
                             precision="f32")


def test_bytes_model_per_pass():
    # 2 q (N - 1) value sizes per node: 56 B per node-component update on D3Q7 FP32, 40 on D2Q5
    assert bench.pass_bytes(HEADLINE) == 22_548_578_304
    assert bench.pass_bytes(TERNARY_2D) == 16_777_216 * 2 * 40
    assert bench.pass_bytes(SimpleNamespace(lattice="D1Q3", N=3, nodes=256, precision="f64")) == 256 * 2 * 48


def test_launch_count_of_blocked_runs():
    r = bench.sweep_record(HEADLINE, 1.0, 500, 2)
    assert r["launches"] == 250 and r["steps_per_pass"] == 2
    assert bench.sweep_record(TERNARY_2D, 1.0, 20, 6)["launches"] == 4    # near-equal passes of at most 6
    assert bench.sweep_record(TERNARY_2D, 1.0, 7, 1)["launches"] == 7


def test_hbm_roofline_while_the_bytes_model_bounds_the_kernel():
    rec = bench.sweep_record(HEADLINE, 500 * 3.155e-3, 500, 2)
    rec.update(per_launch=6.31e-3, per_launch_over="test")
    roof = bench.sweep_roofline(HEADLINE, rec)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["algorithmic_bytes_per_launch"] == 2 * 22_548_578_304
    assert roof["achieved"] == pytest.approx(45_097_156_608 / 6.31e-3 / 1e9, rel=1e-4)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0, abs=1e-4)
    assert roof["frac"] <= 1.0


def test_alu_roofline_past_one_pass_per_launch():
    rec = bench.sweep_record(TERNARY_2D, 2000 * 56e-6, 2000, 6)
    rec.update(per_launch=0.33e-3, per_launch_over="test")
    assert bench.hbm_roofline(TERNARY_2D, rec)["frac"] > 1.0
    roof = bench.sweep_roofline(TERNARY_2D, rec)
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    assert roof["peak"] == pytest.approx(256 * 4 * 16 * 2 * 2.4e9 / 1e12, abs=0.01)
    flops = bench.collision_flops(2, 5) * 16_777_216 * 6
    assert roof["achieved"] == pytest.approx(flops / 0.33e-3 / 1e12, abs=0.01)
    assert 0.0 < roof["frac"] < 1.0


def test_counter_traffic_only_for_the_sources_it_was_measured_on(monkeypatch):
    path = os.path.join(ROOT, "profiles", f"traffic_{HEADLINE.name}.txt")
    vals = dict(ln.split(":", 1) for ln in open(path) if ":" in ln and not ln.startswith("#"))
    vals = {k.strip(): v.strip() for k, v in vals.items()}
    monkeypatch.setattr(bench, "kernel_hash", lambda: vals["kernel_sources_sha256_16"])
    assert bench.load_traffic(HEADLINE.name) == float(vals["hbm_bytes_per_launch"])
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.load_traffic(HEADLINE.name) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
