"""bench.py's host-side contract (no GPU): the multi-GPU request is refused
before anything touches a device, and the measured-traffic figure is reported
only while the contraction sources hash to the value recorded with the
counters."""
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
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = b.contraction_source_hash()
    (prof / "traffic_k_contract_bf16x3_w.md").write_text("x\nsource_sha256: %s\nhbm_bytes_per_launch: 1.5e+10\n" % sha)
    monkeypatch.setattr(b, "contraction_source_hash", lambda: sha)   # the sources as they are now
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("w") == 1.5e10
    assert b.measured_traffic("absent") is None
    monkeypatch.setattr(b, "contraction_source_hash", lambda: "0" * 64)
    assert b.measured_traffic("w") is None
