"""The C-ABI library loads and exports every function include/qtraj.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtraj.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:qt_status|const char\*)\s+(qt_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def qtlib():
    from paper_2107_06147_amd import qtraj
    if not os.path.exists(qtraj.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return qtraj


def test_header_declares_the_api():
    names = declared()
    assert "qt_run" in names and "qt_submit" in names and len(names) >= 20


def test_every_declared_symbol_is_exported(qtlib):
    lib = ctypes.CDLL(qtlib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps exactly those
    assert sorted(qtlib.SYMBOLS) == declared()


def test_version_and_error_without_gpu(qtlib):
    L = qtlib.lib()
    assert b"gfx950" in L.qt_version()
    assert isinstance(L.qt_last_error(), bytes)
    # a null context is rejected without touching the device
    assert L.qt_run(None, None, None, None, None, None, None) == qtlib.QT_EINVAL
    assert b"null" in L.qt_last_error()


def test_oracle_and_library_share_no_code():
    """The GPU library's sources never include or name the oracle, and the
    oracle never includes the library's headers."""
    csrc = os.path.join(ROOT, "paper_2107_06147_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("qtraj_oracle.c", "qtraj_oracle.h"):
        txt = open(os.path.join(ROOT, "oracle", f)).read()
        assert "qtraj.h" not in txt and "qt_internal" not in txt and "csrc" not in txt
    for f in ("qtraj.py", "__init__.py", "build.py"):
        txt = open(os.path.join(ROOT, "paper_2107_06147_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, f
