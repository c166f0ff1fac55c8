"""The C-ABI library loads without a GPU and exports what include/tvd.h declares."""
import ctypes
import os
import re

import pytest

from paper_0907_3390_amd import tvd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tvd.LIB_PATH):
        from paper_0907_3390_amd import build
        build.build()
    return tvd.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tvd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tvd_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(tvd.EXPORTS) == set(names)


def test_status_strings(lib):
    assert tvd.status_string(tvd.TVD_OK) == "ok"
    assert "overlap" in tvd.status_string(tvd.TVD_ERR_ALIAS)
    assert tvd.status_string(12345) == "unknown status"


def test_null_context_is_rejected_before_any_device_call(lib):
    b = tvd.tvd_batch(tvd.TVD_F32, 1, 8, 0, None, None, None, None, None, 1e-3, 1.0)
    st = lib.tvd_patch_advance(None, ctypes.byref(b), None, None, 0, 5 / 3, 0.0, 0, None, None, None)
    assert st == tvd.TVD_ERR_INVALID_ARG
    assert lib.tvd_destroy(None) == tvd.TVD_ERR_INVALID_ARG
    assert lib.tvd_create(None, 0) == tvd.TVD_ERR_INVALID_ARG
    assert lib.tvd_last_error(None) == b""


def test_header_documents_every_entry_point():
    """Each declaration in the header is preceded by a comment."""
    src = open(os.path.join(ROOT, "include", "tvd.h")).read()
    for n in declared_functions():
        m = re.search(r"^(?:int|const char \*)\s*" + n + r"\(", src, flags=re.M)
        assert m, n
        before = src[:m.start()].rstrip()
        assert before.endswith("*/") or before.endswith(";"), n
        assert "*/" in src[max(0, m.start() - 800):m.start()], n
