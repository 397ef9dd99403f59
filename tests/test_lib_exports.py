"""The C-ABI library loads without a GPU and exports every function the
header declares; the binding's signature table covers the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhesql.h")
LIB = os.path.join(ROOT, "paper_2510_15413_amd", "libfhesql.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_hot_path_calls():
    names = declared()
    for must in ("tfhe_bootstrap_batch", "tfhe_keyswitch_batch", "sql_mask_scan", "sql_masked_select",
                 "sql_masked_sum", "sql_scan_batch", "sql_server_step", "sql_radix_mask_scan"):
        assert must in names
    assert len(names) >= 30


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2510_15413_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2510_15413_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(_lib.FheError):
        _lib.load()
