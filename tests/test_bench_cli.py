"""Host logic of bench.py that needs no GPU: the multi-GPU request is refused
with a message (the build covers one GPU), and the traffic record is read
only while the smoother's sources match its digest."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_follows_the_sources(tmp_path, monkeypatch):
    b = _bench()
    # a record for other sources is ignored
    rec = tmp_path / "traffic.md"
    rec.write_text("- traffic_bytes_per_launch: `123`\n- source_digest: `0000000000000000`\n")
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(rec))
    assert b.measured_traffic() is None
    rec.write_text(f"- traffic_bytes_per_launch: `123`\n- source_digest: `{b.kernel_source_digest()}`\n")
    assert b.measured_traffic() == 123.0
