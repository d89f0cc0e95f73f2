"""Host logic of bench.py, without a device: the error measures attached to
every result, the HIP kernel named for each fine variant, the counter-traffic
lookup that is void once the kernel source changes, and the refusal of a run
on more than one GPU.  CPU only."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_error_measures():
    r = np.array([3.0, 4.0, 0.0, 0.0])
    d = np.array([0.0, -0.5, 0.25, 0.0])
    e = bench.errs(r + d, r)
    assert e["max_abs"] == 0.5
    # relative L2 = |d| / |r|, reported to three significant digits
    assert e["rel_l2"] == pytest.approx(np.sqrt(0.25 + 0.0625) / 5.0, rel=1e-3)
    assert bench.errs(r - d, r) == e
    assert bench.errs(r, r) == {"max_abs": 0.0, "rel_l2": 0.0}


@pytest.mark.parametrize("name,kernel", [
    ("rk4w_f64_x128_y8_p2x1_w16", "rk4_step_rows"),
    ("rk4s_f64_x32_y32_p2x1_w10", "rk4_step_rows"),
    ("rk4x_f32_t56x40_p1x3_w16", "rk4_step_rows"),
    ("rk4b_f32_t64x32_p2x2_d2", "rk4_step_fused1b"),
    ("rk4r_f32_o4_t32x16_p2x2_d2", "rk4_step_fused1r"),
    ("rk4h_f64_o4_x128_y8_p2_w16_d1", "rk4_half_rows"),
    ("rk4hx_f64_o4_t120x8_p2_w16_d1", "rk4_half_rows"),
    ("rk4_f32_o4_t32x16_p1x2", "rk4_step_fused"),
    ("rk4_unfused_reference", "rk4_stage_ref"),
])
def test_kernel_of(name, kernel):
    assert bench.kernel_of(name) == kernel


def test_every_registered_fine_variant_names_a_fused_kernel():
    import paper_1409_8563_amd as pr
    names = [v["name"] for v in pr.variants(0)]
    assert names
    for n in names:
        assert bench.kernel_of(n) != "rk4_stage_ref", n
    # the two-launch fourth-order pairs are the only half-step kernels
    for v in pr.variants(0):
        if bench.kernel_of(v["name"]) == "rk4_half_rows":
            assert v["order"] == 4 or v["name"].startswith("rk4h_f32"), v["name"]


def _fake_record(tmp_path, source_text, per_launch):
    src = tmp_path / "stencil_kernels.hip"
    src.write_text(source_text)
    rec = {"stencil_kernels_sha256": hashlib.sha256(source_text.encode()).hexdigest(),
           "summary": "profiles/x.md", "per_launch_bytes": per_launch}
    js = tmp_path / "hbm_traffic.json"
    js.write_text(json.dumps(rec))
    return src, js


def test_traffic_lookup_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    src, js = _fake_record(tmp_path, "// kernels v1\n", {"rk4w_a@c2": 123456})
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(js))
    v, note = bench.measured_traffic("rk4w_a", "c2")
    assert v == 123456 and "FETCH_SIZE" in note
    assert bench.measured_traffic("rk4w_a", "c3")[0] is None         # other workload
    assert bench.measured_traffic("rk4w_b", "c2")[0] is None         # other variant
    src.write_text("// kernels v2\n")                                 # source edited after the counters
    v, note = bench.measured_traffic("rk4w_a", "c2")
    assert v is None and "changed" in note
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("rk4w_a", "c2")[0] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
