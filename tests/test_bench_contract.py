"""bench.py's JSON contract pieces that run without a GPU: the HBM traffic
figure is taken from the committed counter summary only while the march
sources hash to the value recorded there, and multi-GPU runs are refused."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    good = tmp_path / "traffic.md"
    good.write_text("traffic_bytes_per_launch: 123456\n\nmarch_sources_sha256: `%s`\n"
                    % bench.march_sources_sha256())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic() == 123456
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 123456\n\nmarch_sources_sha256: `%s`\n" % ("0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_march_source_hash_covers_the_march_kernel_files():
    csrc = os.path.join(ROOT, "paper_2309_04581_amd", "csrc")
    for f in bench.MARCH_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    assert "march_mfma.hip" in bench.MARCH_SOURCES and "mr_mfma.h" in bench.MARCH_SOURCES


def test_committed_traffic_summary_is_parseable():
    with open(bench.TRAFFIC_FILE) as fh:
        text = fh.read()
    assert "traffic_bytes_per_launch:" in text and "march_sources_sha256:" in text


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_work_per_sample():
    from paper_2309_04581_amd import scenegen as sg
    f = sg.mid_field()
    # density 32x64 + 64x16, colour (16+16)x64 + 64x64 + 3x64
    assert bench.field_macs(f) == 32 * 64 + 64 * 16 + 32 * 64 + 64 * 64 + 3 * 64 == 9408
    assert bench.gather_bytes(f) == 16 * 8 * 2 * 4 == 1024
