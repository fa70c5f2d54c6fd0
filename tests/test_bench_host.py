"""Host-side pieces of bench.py that need no GPU: the single-GPU guard, the
algorithmic byte count of a colour pass, and the reading of the committed
HBM counter summary (taken only while the kernel sources it was measured on
are unchanged)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_a_pass():
    # read both colours and write one: 3 components each, 4 or 8 bytes
    n = 256 ** 3
    assert bench.algorithmic_pass_bytes(n, 32) == 36 * (n // 2) == 301989888
    assert bench.algorithmic_pass_bytes(n, 64) == 72 * (n // 2)
    assert bench.algorithmic_pass_bytes(384 ** 3, 32) == 1019215872


def _summary(tmp_path, sha):
    p = tmp_path / "traffic.md"
    p.write_text("# counters\n\nsome text: 12\n\n"
                 f"source_sha256: {sha}\n"
                 "pass_fetch_kib_per_dispatch: 100.0\n"
                 "pass_write_kib_per_dispatch: 50.0\n"
                 "copy_fetch_scale: 2.0\n"
                 "copy_write_scale: 1.0\n")
    return str(p)


def test_traffic_summary_is_read_while_the_sources_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, bench.kernel_source_hash()))
    assert bench.measured_traffic(0) == (100.0 * 2.0 + 50.0 * 1.0) * 1024.0


def test_traffic_summary_is_dropped_once_the_sources_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, "0000000000000000"))
    assert bench.measured_traffic(0) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic(0) is None


def test_committed_summary_is_well_formed():
    # the committed summary parses, whatever the state of the sources
    text = open(bench.TRAFFIC_FILE).read()
    for key in ("source_sha256", "pass_fetch_kib_per_dispatch", "pass_write_kib_per_dispatch",
                "copy_fetch_scale", "copy_write_scale"):
        assert f"\n{key}: " in text, key
