"""CPU tests of the bench's HBM-traffic lookup: counter values are scaled by
the copy calibration and reported only while the kernel source still has the
hash the counters were taken on."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, src_text, sha=None, rows=((14, 1000.0, 2000.0),)):
    src = tmp_path / "kernels.hip"
    src.write_text(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    lines = ["# comment", "kernel_source_sha256 " + digest, "fetch_factor 2.0000", "write_factor 1.0000"]
    lines += ["tiling %d fetch_kib %.1f write_kib %.1f   # note" % r for r in rows]
    pmc = tmp_path / "pmc.txt"
    pmc.write_text("\n".join(lines) + "\n")
    return str(src), str(pmc)


def test_traffic_is_scaled_counter_bytes(tmp_path, monkeypatch):
    src, pmc = _write(tmp_path, "kernel v1")
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PMC_FILE", pmc)
    assert bench.sweep_traffic(14) == (1000.0 * 2.0 + 2000.0 * 1.0) * 1024.0


def test_changed_kernel_source_gives_no_traffic(tmp_path, monkeypatch):
    src, pmc = _write(tmp_path, "kernel v1", sha=hashlib.sha256(b"kernel v0").hexdigest())
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PMC_FILE", pmc)
    assert bench.sweep_traffic(14) is None


def test_unprofiled_tiling_or_missing_file_gives_no_traffic(tmp_path, monkeypatch):
    src, pmc = _write(tmp_path, "kernel v1")
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PMC_FILE", pmc)
    assert bench.sweep_traffic(3) is None
    monkeypatch.setattr(bench, "PMC_FILE", str(tmp_path / "absent.txt"))
    assert bench.sweep_traffic(14) is None
