"""CPU checks of the C-ABI boundary: the library builds, loads and exports
every entry point that include/fraclap.h declares (no device calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fraclap.h")
SO = os.path.join(ROOT, "paper_1911_11906_amd", "libfraclap.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        from paper_1911_11906_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(SO)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fl_assemble", "fl_eigensolve", "fl_apply_fractional", "fl_grad_apply"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_binding_covers_every_declared_symbol():
    from paper_1911_11906_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", SO], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(fl_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1911_11906_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved
