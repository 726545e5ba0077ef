"""Host-side checks of the benchmark script: the one-GPU contract and its roofline arithmetic."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_picks_the_binding_roof():
    # FP32 at 64 RHS: 2*F*64 flops against 4*F bytes is above the FP32 ridge -> MFMA-bound
    F, n, m = 10**8, 65536, 16384
    r = bench.roofline_for("f32", F, n, m, 64, apply_ms=1.0, launches=11)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - 2.0 * F * 64 / 1e-3 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 157.3) < 1e-12
    # one RHS: bytes dominate -> HBM-bound, algorithmic bytes = 4 F + 4 (n + m)
    r1 = bench.roofline_for("f32", F, n, m, 1, apply_ms=1.0, launches=11)
    assert r1["bound"] == "hbm"
    assert abs(r1["achieved"] - (4.0 * F + 4.0 * (n + m)) / 1e-3 / 1e9) < 1e-6
    # split products multiply the executed flops
    r3 = bench.roofline_for("bf16x3", F, n, m, 256, apply_ms=1.0, launches=11)
    assert r3["bound"] == "mfma" and abs(r3["achieved"] - 6 * 2.0 * F * 256 / 1e-3 / 1e12) < 1e-6


def test_level_bytes_counts_every_level_vector_twice():
    fs = {"L": 1, "rank": np.array([[1, 2], [3, 4]], dtype=np.int32), "ident": np.zeros((2, 2), np.uint8)}
    assert bench.folded_levels(fs) == 0
    assert bench.level_bytes(fs, 8, 4) == 2.0 * 10 * 8 * 4
    # a leading all-identity level is folded: it has no level vector of its own
    fs["ident"][0] = 1
    assert bench.folded_levels(fs) == 1
    assert bench.level_bytes(fs, 8, 4) == 2.0 * 7 * 8 * 4


def test_merged_plans_form_no_last_level_vector():
    # with the leaf bases merged into the last level, y_L is never written
    fs = {"L": 1, "rank": np.array([[1, 2], [3, 4]], dtype=np.int32), "ident": np.zeros((2, 2), np.uint8)}
    assert bench.level_bytes(fs, 8, 4, merged=True) == 2.0 * 3 * 8 * 4


def test_counter_records_follow_their_sources(tmp_path, monkeypatch):
    """A counter record counts only while every source it lists has the hash it
    was taken with; a record that lists no sources never counts."""
    import hashlib
    import json
    src = tmp_path / "src" / "k.hip"
    src.parent.mkdir()
    src.write_text("kernel v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sources_sha1": {"src/k.hip": hashlib.sha1(b"kernel v1\n").hexdigest()},
           "fwd": {"hbm_bytes_per_launch": 5.0, "hbm_bytes_per_apply": 35.0}, "fwd_mfma": {"mfma_busy_pct": 40.0}}
    (prof / "hbm_traffic_w.json").write_text(json.dumps(rec))
    (prof / "hbm_traffic_old.json").write_text(json.dumps({"kernels_hip_sha1": "x", "fwd": rec["fwd"]}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w") == 5.0 and bench.measured_traffic("w", per="apply") == 35.0
    assert bench.measured_mfma_busy("w") == 40.0
    assert bench.measured_traffic("old") is None and bench.measured_traffic("missing") is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("w") is None and bench.measured_mfma_busy("w") is None


def test_stage_launches_follow_the_plan():
    """Launches per apply come from the plan: L + 1 stages with merged leaf
    blocks, L + 2 with the separate leaf stage, less the folded levels."""
    from types import SimpleNamespace
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from factor_gen import random_factor_set
    from paper_2605_21828_amd import bfmht as B
    fs = random_factor_set(31, 600, 256, 4, max_rank=40, ident_levels=1, p_id_form=0.5, full_rank_leaves=True)
    assert bench.folded_levels(fs) == 1
    for flags, stages in ((0, 5), (B.PLAN_LEAF_STAGE, 6)):
        h = B.bfmht_plan_create_ex(fs, B.F32, 4, flags)
        try:
            assert bench.stage_launches(SimpleNamespace(handle=h), fs) == stages - 1
        finally:
            B.bfmht_plan_destroy(h)
