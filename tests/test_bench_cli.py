"""Host logic of bench.py that needs no GPU: the multi-GPU request is refused
with a message (the build covers one GPU), and the defaults name the
power-law workload with FP64 cycles."""
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


def test_default_workload_is_the_power_law_graph_in_fp64(monkeypatch):
    b = _bench()
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = b.parse()
    assert a.workload == "powerlaw" and a.cycle_prec is None and a.n0 == 4_000_000 and a.gpus == 1
    # the flush between timed passes exceeds the 256 MB last-level cache
    assert b.FLUSH_BYTES >= 4 * (256 << 20)


def test_traffic_record_follows_the_sources(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter record only while the
    kernel sources it names are unchanged (digest of their bytes)."""
    import hashlib
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    rec = tmp_path / "rec.md"
    rec.write_text(f"- traffic_bytes_per_launch: `1234`\n- source_digest: `{digest}`\n- sources: `{src}`\n")
    monkeypatch.setattr(b, "TRAFFIC_RECORD", str(rec))
    monkeypatch.setattr(b, "ROOT", "/")
    assert b.traffic_record() == 1234
    src.write_text("kernel v2\n")
    assert b.traffic_record() is None
