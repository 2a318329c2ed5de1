"""The C-ABI library loads and exports every entry point include/polymh.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_16576_amd", "libpolymh.so")
HDR = os.path.join(ROOT, "include", "polymh.h")


def declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polymh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("polymh_sign", "polymh_band", "polymh_query", "polymh_refine"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpolymh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpolymh.so not built")
def test_binding_covers_every_declared_symbol():
    from paper_2511_16576_amd import polymh as pm
    assert set(declared()) <= set(pm._SIGNATURES)
    pm.lib()


def test_library_and_oracle_share_no_code():
    csrc = os.path.join(ROOT, "paper_2511_16576_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2511_16576_amd" not in text and "polymh.h" not in text, f
