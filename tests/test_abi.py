"""The C-ABI library loads and exports every entry point include/he.h declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_hot_path_calls():
    names = declared_functions()
    for n in ["he_ntt", "he_rotate", "he_rotate_hoisted", "he_mul_plain", "he_relin", "he_conv2d",
              "he_avgpool", "he_fc"]:
        assert n in names, n


def test_library_exports_every_declared_symbol():
    from paper_2510_03996_amd import he

    lib = ctypes.CDLL(he.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2510_03996_amd import he

    monkeypatch.setattr(he, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(he, "_lib", None)
    try:
        he.lib()
    except RuntimeError as e:
        assert "not built" in str(e)
    else:
        raise AssertionError("expected a loud failure")
