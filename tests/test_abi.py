"""The C ABI library loads and exports every entry point include/eofa.h declares (CPU-side)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "eofa.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eofa_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    from paper_1710_09621_amd import eofa as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("libeofa.so not built")
    lib = ctypes.CDLL(E.LIB_PATH)
    names = declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_without_gpu():
    import torch
    from paper_1710_09621_amd import eofa as E
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        E.Context((4, 4, 4, 4), 8, 1.3, [1.0] * 8)
