"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU oracle
and of the library's host code, each driven through its code paths by a
small program (tests/sanitize/).  The device code of the library is built
as usual; only its host side is instrumented.  No GPU is needed: the host
driver exercises argument validation and error paths, the oracle driver
runs every lattice, boundary, force, scheme and model for a few steps."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-ffp-contract=off", "-o", exe, os.path.join(ROOT, "oracle", "vflb_oracle.c"),
                    os.path.join(SAN, "oracle_driver.c"), "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver: ok" in r.stdout


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_2506_13072_amd", "csrc")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
                    "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-o", exe,
                    os.path.join(csrc, "vflb.hip"), os.path.join(csrc, "mlp.hip"),
                    os.path.join(SAN, "host_driver.cpp")], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host driver: 0 unexpected" in r.stdout
