"""Host-side logic of bench.py (no GPU): the one-GPU guard, the attempts
histogram, and the rule that committed counters count only for the kernel
sources they were taken on."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_attempts_histogram():
    b = load_bench()
    att = np.array([1, 2, 3, 201, 230, 255, 256, 780])
    h = b.attempts_histogram(att)
    assert h["p0"] == 1.0 and h["p100"] == 780.0
    assert h["log2_bins"] == {"0": 1, "1": 2, "7": 3, "8": 1, "9": 1}
    assert sum(h["log2_bins"].values()) == att.size


def test_counters_only_for_matching_sources(tmp_path, monkeypatch):
    b = load_bench()
    good = {"source_sha256": b.kernel_source_hash(), "fetch_bytes": 1.0, "write_bytes": 2.0,
            "launch": "256,2,1,8,3", "executed_fp64_flop": 5.0}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(good))
    monkeypatch.setattr(b, "COUNTER_FILE", str(f))
    assert b.committed_counters()["executed_fp64_flop"] == 5.0
    f.write_text(json.dumps(dict(good, source_sha256="0" * 64)))
    assert b.committed_counters() is None
    monkeypatch.setattr(b, "COUNTER_FILE", str(tmp_path / "missing.json"))
    assert b.committed_counters() is None


def test_gate_stats_ignore_failed_rays():
    b = load_bench()
    o = {"cls": np.array([0, 1, 2, 0]), "h_gate": np.array([1e-9, 5e-9, 1.0, 2e-9])}
    g = b.gate_stats(o)
    assert g["holds"] and g["failed_rays"] == 1 and g["h_gate_max"] == 5e-9 and g["frac_le_1e-8"] == 1.0
    o["h_gate"][3] = 2e-8
    g = b.gate_stats(o)
    assert not g["holds"] and g["frac_le_1e-8"] == 2 / 3


def test_gate_tolerances_are_the_listed_ones():
    b = load_bench()
    assert b.GATE_RTOLS == (1e-8, 3e-9, 1e-9, 3e-10, 1e-10)
    assert max(b.GATE_RTOLS_BEYOND) < min(b.GATE_RTOLS)
    s = b.solver_at({"solver": {"rtol": 1e-8, "atol": 1e-10, "r_escape": 1100.0}}, 3e-10)
    assert s["rtol"] == 3e-10 and s["atol"] == 3e-12


def test_gather_roofline_counts_six_rhs_per_attempt_and_one_per_ray():
    b = load_bench()
    rec = {"attempts_per_ray": 10.0, "kernel_ms": 2.0}
    g = b.gather_roofline(rec, 1000)
    rhs = 10.0 * 1000 * 6 + 1000
    assert g["rhs_per_launch"] == rhs
    assert abs(g["achieved"] - rhs * 640 / 2e-3 / 1e12) < 1e-12
    assert abs(g["frac"] - g["achieved"] / g["peak"]) < 1e-15
    assert abs(g["peak"] - 8 * 16 * 128 * 2.4e9 / 1e12) < 1e-9
