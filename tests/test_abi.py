"""The C-ABI library loads and exports every symbol include/bem.h declares (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_documented_entry_points():
    syms = declared_symbols()
    for name in ("bem_assemble", "bem_precond_setup", "bem_pcg_solve", "bem_serve_submit", "bem_serve_poll"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2310_09204_amd import lib
    L = ctypes.CDLL(lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    # and the Python binding knows every one of them
    assert set(declared_symbols()) <= set(lib.SIGNATURES)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2310_09204_amd import lib
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(RuntimeError):
        lib.load()
