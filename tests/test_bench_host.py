"""Host-side checks of bench.py (no GPU): the readers of the committed profile
summaries report a figure only for the kernel and sources it was measured on, and a
multi-GPU request is refused with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

W2 = "scf_triaxial_hernquist_n1e6_n10_l10"
FORCE = "scf_force_kernel<float, 10, true, 0>"


def test_counters_follow_the_sources(monkeypatch):
    rec = bench.measured_counters("force", W2, FORCE)
    if rec is None:
        pytest.skip("force kernel sources changed since its counters were taken")
    assert rec["kernel"] == FORCE and rec["units_per_launch"] == 1_000_000
    assert 0.0 < rec["valu_issue_busy"] <= 1.0
    assert rec["valu_instr_per_unit"] > 0 and rec["executed_fp32_flop_per_unit"] > 0
    # another kernel name, or other sources: nothing
    assert bench.measured_counters("force", W2, "scf_force_kernel<float, 10, false, 0>") is None
    monkeypatch.setattr(bench, "source_digest", lambda which: "0" * 64)
    assert bench.measured_counters("force", W2, FORCE) is None
    assert bench.measured_traffic("force", W2) is None


def test_missing_summaries_give_nothing():
    assert bench.measured_counters("force", "no_such_workload", FORCE) is None
    assert bench.measured_traffic("force", "no_such_workload") is None


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "single" in (r.stdout + r.stderr).lower()
