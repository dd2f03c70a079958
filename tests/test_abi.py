"""The C-ABI library loads, exports every entry point its header declares,
and validates arguments on the host (no GPU needed for these calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vflb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vflb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2506_13072_amd import vflb
    return vflb.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("vflb_create", "vflb_bind_buffers", "vflb_set_params", "vflb_set_force",
              "vflb_set_boundaries", "vflb_init_fields", "vflb_step", "vflb_reduce",
              "vflb_read", "vflb_save", "vflb_load", "vflb_destroy", "vflb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    path = os.path.join(ROOT, "paper_2506_13072_amd", "libvflb.so")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(vflb_\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(lib, n)


def test_create_validates_arguments_on_host(lib):
    h = ctypes.c_void_p()
    assert lib.vflb_create(7, 8, 8, 1, 1, None, ctypes.byref(h)) == 1   # lattice
    assert b"lattice" in lib.vflb_last_error(None)
    assert lib.vflb_create(2, 8, 8, 1, 9, None, ctypes.byref(h)) == 1   # storage
    assert lib.vflb_create(2, 0, 8, 1, 1, None, ctypes.byref(h)) == 1   # size
    assert lib.vflb_create(3, 8, 8, 0, 1, None, ctypes.byref(h)) == 1
    assert not h.value


def test_create_rejects_sizes_and_options_not_built(lib):
    h = ctypes.c_void_p()
    mk = lambda *a: lib.vflb_create_ex(*a, None, ctypes.byref(h))
    # D3Q19 node limits of the 32-bit plane offsets: 2^26 FP64, 2^27 FP32,
    # 2^28 16-bit
    assert mk(3, 512, 512, 257, 0, 0, 0) == 1
    assert mk(3, 512, 512, 513, 1, 0, 0) == 1
    assert mk(3, 1024, 512, 513, 2, 0, 0) == 1
    assert b"exceeds" in lib.vflb_last_error(None)
    assert mk(2, 8, 8, 1, 1, 0, 2) == 1              # unknown option bit
    assert mk(3, 8, 8, 8, 2, 0, 1) == 1              # in place: not 16-bit
    assert mk(2, 8, 8, 1, 2, 0, 1) == 1              # in place: not 16-bit
    assert mk(3, 8, 8, 8, 2, 1, 0) == 1              # comparison scheme: not 16-bit
    assert mk(2, 8, 8, 1, 1, 5, 0) == 1              # unknown scheme
    assert mk(3, 16, 16, 16, 3, 0, 0) == 1           # BF16 storage on D3Q19
    assert b"BF16" in lib.vflb_last_error(None)
    assert not h.value


def test_python_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2506_13072_amd import vflb
    monkeypatch.setattr(vflb, "_lib", None)
    monkeypatch.setattr(vflb, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        vflb.lib()


def test_batch_create_validates_arguments_on_host(lib):
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 6)(64, 64, 1, 32, 16, 1)
    lib.vflb_batch_last_error.restype = ctypes.c_char_p
    assert lib.vflb_batch_create(3, 2, dims, 1, None, ctypes.byref(h)) == 1   # D3Q19
    assert b"D2Q9" in lib.vflb_batch_last_error(None)
    assert lib.vflb_batch_create(2, 0, dims, 1, None, ctypes.byref(h)) == 1   # empty
    assert lib.vflb_batch_create(2, 2, None, 1, None, ctypes.byref(h)) == 1   # no dims
    assert lib.vflb_batch_create(2, 2, dims, 7, None, ctypes.byref(h)) == 1   # storage
    bad = (ctypes.c_int * 6)(64, 64, 1, 0, 16, 1)
    assert lib.vflb_batch_create(2, 2, bad, 1, None, ctypes.byref(h)) == 1    # size
    assert b"instance 1" in lib.vflb_batch_last_error(None)
    assert not h.value


def test_copy_probe_validates_arguments_on_host(lib):
    P = ctypes.c_void_p
    assert lib.vflb_copy_probe(P(16), P(32), 32, 4, None) == 1          # kind
    assert b"kind" in lib.vflb_last_error(None)
    assert lib.vflb_copy_probe(P(16), P(32), 24, 1, None) == 1          # 16-byte size
    assert lib.vflb_copy_probe(P(8), P(32), 32, 3, None) == 1           # alignment
    assert lib.vflb_copy_probe(P(16), P(32), 0, 2, None) == 0           # empty: no launch
    assert lib.vflb_stream_copy(P(16), P(32), 17, None) == 1
