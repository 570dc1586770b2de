"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sqd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sqd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    from paper_2601_16169_amd import sqd
    assert set(declared_functions()) == set(sqd.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2601_16169_amd import sqd
    if not os.path.exists(sqd.LIB_PATH):
        pytest.skip("libsqd.so not built")
    lib = ctypes.CDLL(sqd.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    assert lib.sqd_version  # callable without a device
    lib.sqd_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.sqd_version()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2601_16169_amd import sqd
    monkeypatch.setattr(sqd, "_lib", None)
    monkeypatch.setattr(sqd, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        sqd.lib()


def test_product_does_not_import_oracle():
    """No module of the product package refers to the oracle."""
    pkg = os.path.join(ROOT, "paper_2601_16169_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
