"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_dropped_when_kernels_change(tmp_path, monkeypatch):
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    h = b.kernel_source_hash()
    assert len(h) == 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_stage_demo_traffic.md").write_text(
        f"traffic_bytes_per_launch: 123.0\nsource_sha256: `{h}`\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    # sources are read from ROOT too: point them back at the real tree
    monkeypatch.setattr(b, "kernel_source_hash", lambda: h)
    assert b.measured_traffic("demo", "k_stage") == 123.0
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 64)
    assert b.measured_traffic("demo", "k_stage") is None


def test_exchange_interval_follows_the_ghost_layers():
    import importlib.util
    import pytest
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    muscl_rk2 = dict(scheme=1, integrator=1)
    waf = dict(scheme=2, integrator=0)
    hllc1 = dict(scheme=0, integrator=0)
    assert b.exchange_interval(muscl_rk2, 4) == 1
    assert b.exchange_interval(waf, 4) == 2
    assert b.exchange_interval(hllc1, 4) == 4
    assert b.exchange_interval(hllc1, 4, requested=1) == 1
    assert b.exchange_interval(dict(scheme=1, integrator=0), 4) == 2
    with pytest.raises(SystemExit):
        b.exchange_interval(waf, 4, requested=3)
