"""CPU checks of bench.py's host logic: the one-GPU guard, and the reading of
the committed counter summaries (used only while the solve-kernel sources
still hash the same as when the counters were taken)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_summaries_follow_the_source_hash(tmp_path, monkeypatch):
    b = _bench()
    h = b.solve_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    valu = tmp_path / "valu.txt"
    valu.write_text("header line\nvalu row 0.8672 issue_frac source %s\nvalu col 0.7146 issue_frac source 0123\n" % h)
    traffic = tmp_path / "traffic.txt"
    traffic.write_text("traffic row 360393049 bytes_per_launch source %s\n" % h)
    monkeypatch.setattr(b, "VALU_FILE", str(valu))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(traffic))
    assert b.measured_valu_issue("row") == 0.8672
    assert b.measured_valu_issue("col") is None  # taken on other sources
    assert b.measured_traffic("row") == 360393049.0
    assert b.measured_traffic("col") is None
    monkeypatch.setattr(b, "solve_source_hash", lambda: "ffffffffffffffff")
    assert b.measured_valu_issue("row") is None and b.measured_traffic("row") is None
    monkeypatch.setattr(b, "VALU_FILE", str(tmp_path / "missing.txt"))
    assert b.measured_valu_issue("row") is None
