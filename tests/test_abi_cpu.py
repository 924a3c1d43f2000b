"""The C-ABI library loads and exports every entry point include/mpsvqe.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpsvqe.h")
LIB = os.path.join(ROOT, "paper_2211_07983_amd", "libmpsvqe.so")


def declared():
    text = open(HEADER).read()
    decl = r"^\s*(?:mps_status|void|const char\s*\*|int64_t|int32_t)\s+(mps_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_header_declares_the_four_operations():
    names = declared()
    for op in ("mps_init_product", "mps_apply_circuit", "mps_expect_paulisum", "mps_energy_grad"):
        assert op in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_header_exports():
    from paper_2211_07983_amd import _abi
    assert sorted(_abi.EXPORTS) == declared()


def test_binding_refuses_missing_library(tmp_path):
    from paper_2211_07983_amd import _abi
    old = _abi._lib
    _abi._lib = None
    try:
        with pytest.raises(ImportError):
            _abi.load(str(tmp_path / "nope.so"))
    finally:
        _abi._lib = old
