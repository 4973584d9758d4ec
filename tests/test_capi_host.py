"""Host-only checks of the C-ABI library: it loads and exports every function
that include/nosdd.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_2509_03622_amd import nosdd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nosdd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nosdd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert set(_declared()) == set(nosdd.EXPORTS)


@pytest.mark.skipif(not os.path.exists(nosdd.LIBPATH), reason="libnosdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(nosdd.LIBPATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(nosdd.LIBPATH), reason="libnosdd.so not built")
def test_null_handles_are_accepted_by_destroy_and_rejected_elsewhere():
    L = nosdd.load()
    L.nosdd_ctx_destroy(None)
    L.nosdd_problem_destroy(None)
    assert L.nosdd_last_error(None) == b"null context"
    assert L.nosdd_ctx_create(0, None, None) == -1
    assert L.nosdd_tile_info(None, 0, None) == -1
    assert L.nosdd_sizes(None, None, None, None, None) == -1
    assert L.nosdd_last_timing(None, None, None, None) == -1
