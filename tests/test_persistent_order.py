"""The work order of the persistent batched apply, replayed on the CPU.

Compiles tests/native/sched_sim.cpp with the library's own scheduling header
(paper_2605_21828_amd/csrc/persistent_sched.h, no HIP) and runs it: every
item's dependency is listed earlier in every queue, replays with one to three
resident workgroups per queue (far fewer than the items) and random
interleavings always finish, and a planted reversed order deadlocks in the
replay (so the replay can see a deadlock)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_persistent_work_order_cannot_deadlock(tmp_path):
    exe = str(tmp_path / "sched_sim")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2605_21828_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "sched_sim.cpp"), "-o", exe], check=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    lines = r.stdout.split("\n")
    assert r.returncode == 0, r.stdout + r.stderr
    assert any(l.startswith("ok dependencies") for l in lines)
    assert any(l.startswith("ok replay") for l in lines)
    assert any(l.startswith("ok reversed order deadlocks") for l in lines)
