"""Host-side checks of bench.py: the algorithmic bytes per lattice update it
prices the roofline with, its refusal of more than one GPU, and how it reads
measured traffic from the rocprofv3 records under profiles/."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("d,storage,expected", [
    (2, "f32", 2 * 9 * 4 * 4 + 2 * 5 * 4),        # 36 populations r/w, chi and u r/w
    (2, "f64", 2 * (2 * 9 * 4 * 4 + 2 * 5 * 4)),
    (2, "f16s", 2 * 9 * 4 * 2 + 2 * 5 * 4 + 2 * 24),  # + the FP32 anchor r/w
    (3, "f32", 2 * 19 * 7 * 4 + 2 * 9 * 4),      # 133 populations
    (3, "f16s", 2 * 19 * 7 * 2 + 2 * 9 * 4 + 2 * 40),
])
def test_bytes_per_lattice_update(d, storage, expected):
    assert bench.bytes_per_lup(d, storage) == expected


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _record(path, sha, fetch, write):
    with open(path, "w") as fh:
        fh.write("# record\n\n"
                 f"    sources_sha256: {sha}\n"
                 f"    fetch_bytes_per_launch: {fetch}\n"
                 f"    write_bytes_per_launch: {write}\n")


def test_measured_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    from paper_2506_13072_amd.build import kernel_sources_sha
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    _record(tmp_path / "now.md", kernel_sources_sha("step2d"), 1.5e9, 1.25e9)
    _record(tmp_path / "old.md", "0" * 64, 1.5e9, 1.25e9)
    assert bench.measured_traffic("now.md", "step2d") == 2.75e9
    assert bench.measured_traffic("old.md", "step2d") is None
    # the same record does not describe the other step kernel
    assert bench.measured_traffic("now.md", "step3d") is None
    assert bench.measured_traffic("missing.md", "step2d") is None


@pytest.mark.parametrize("record", [
    "step2d_f32_channel_8192x1024.md",
    "step2d_f16_channel_8192x1024.md",
    "step3d_f16_tgv_512.md",
    "batch2d_f32_ensemble_256.md",
    "aa_step_f32_channel_8192x1024.md",
    "aa_velocity_f32_channel_8192x1024.md",
    "step3d_f32_tgv_512.md",
])
def test_committed_records_are_readable(record):
    # every record bench.py reads carries the machine-read lines it parses
    with open(os.path.join(bench.PROFILES, record)) as fh:
        text = fh.read()
    for key in ("sources_sha256:", "fetch_bytes_per_launch:", "write_bytes_per_launch:",
                "avg_launch_ns:"):
        assert key in text, (record, key)
