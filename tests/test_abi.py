"""CPU checks of the C ABI: the library loads and exports every symbol the header declares.
No compute call is made here."""
import ctypes
import os
import re

import pytest

import paper_2104_04895_amd as fp4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fp4.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fp4_[a-z0-9_]+)\s*\(", text)))


def test_header_lists_the_binding_names():
    assert _declared() == sorted(fp4.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fp4.LIB_PATH):
        pytest.skip("libfp4.so not built")
    L = ctypes.CDLL(fp4.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_strerror_and_null_context():
    if not os.path.exists(fp4.LIB_PATH):
        pytest.skip("libfp4.so not built")
    L = fp4.lib()
    assert L.fp4_strerror(0) == b"success"
    assert L.fp4_strerror(-1) == b"invalid argument"
    assert L.fp4_strerror(-5) == b"unsupported option"
    # every entry point rejects a null context without touching a device
    assert L.fp4_set_param(None, 1, 2.0) == fp4.FP4_E_INVAL
    assert L.fp4_last_stats(None, None, None, None) == fp4.FP4_E_INVAL
    assert L.fp4_last_error(None) == b"null context"
    assert L.fp4_create(None, 0) == fp4.FP4_E_INVAL
    L.fp4_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fp4, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fp4, "_lib", None)
    with pytest.raises(ImportError):
        fp4.Context()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why (no GPU needed)."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
