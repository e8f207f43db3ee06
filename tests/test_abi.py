"""The C-ABI library loads and exports every symbol include/sbie.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

import paper_2506_20809_amd as sbie

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sbie_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_header_declares_the_binding_exports():
    assert _declared_symbols() == set(sbie.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(sbie.LIB_PATH):
        pytest.skip("libsbie.so not built")
    L = ctypes.CDLL(sbie.LIB_PATH)
    missing = [n for n in _declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_without_device():
    if not os.path.exists(sbie.LIB_PATH):
        pytest.skip("libsbie.so not built")
    L = sbie.lib()
    assert L.sbie_status_str(0) == b"ok"
    assert L.sbie_status_str(-8) == b"continued fraction did not converge"


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(sbie, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sbie, "_lib", None)
    with pytest.raises(ImportError):
        sbie.lib()
