"""The C ABI library loads and exports every symbol include/sbv.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sbv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sbv_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for req in ("sbv_build_blocks", "sbv_blocks_import", "sbv_loglik", "sbv_loglik_dev", "sbv_loglik_grad",
                "sbv_loglik_grad_dev", "sbv_last_error"):
        assert req in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2504_12004_amd", "libsbv.so")
    if not os.path.exists(path):
        pytest.fail("libsbv.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_uses_the_c_names():
    from paper_2504_12004_amd import sbv
    for n in _declared():
        if n in ("sbv_last_error",):
            continue
        assert hasattr(sbv, n) or n in ("sbv_fit_opts",), n
