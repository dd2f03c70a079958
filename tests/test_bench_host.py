"""Host-side checks of bench.py: the algorithmic bytes per lattice update it
prices the roofline with, and its refusal of more than one GPU."""
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
