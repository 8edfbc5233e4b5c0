"""Host-side checks of the C ABI library (no GPU needed): it loads and exports every entry point that
include/ap.h declares, the binding names the same set, and context creation errors are reported."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ap.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(ap_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def libap():
    from paper_2512_07693_amd import ap
    if not os.path.exists(ap.LIB_PATH):
        from paper_2512_07693_amd import build as B
        B.build()
    return C.CDLL(ap.LIB_PATH)


def test_every_declared_symbol_is_exported(libap):
    names = _declared()
    assert len(names) >= 12
    for s in names:
        assert hasattr(libap, s), s


def test_binding_covers_the_header():
    from paper_2512_07693_amd import ap
    assert sorted(ap.SYMBOLS) == _declared()


def test_create_rejects_bad_arguments(libap):
    from paper_2512_07693_amd import ap
    L = ap.lib()
    h = C.c_void_p()
    assert L.ap_ctx_create(C.byref(h), 0, 16, 0.5, None) == -1
    assert b"n_max_atoms" in L.ap_last_error(None)
    assert L.ap_ctx_create(C.byref(h), 16, 5000, 0.5, None) == -1
