"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/zm.h, and its pure host functions
(zm_num_moments, zm_index) agree bit-exactly with the oracle's enumeration."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zm.h")
LIB = os.path.join(ROOT, "paper_2304_14492_amd", "libzm.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(zm_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2304_14492_amd import _build  # noqa: F401  (import would raise without the .so)
        pytest.fail("libzm.so missing: build first")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["zm_plan", "zm_plan_ex", "zm_radial_table", "zm_moments", "zm_destroy", "zm_index",
              "zm_num_moments", "zm_plan_info", "zm_workspace_size", "zm_status_str", "zm_last_error"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_exposes_same_names(lib):
    import paper_2304_14492_amd as zm
    assert sorted(zm.exported_symbols()) == sorted(
        n for n in _declared() if n not in ("zm_status_str_",))


def test_index_and_count_match_oracle(lib):
    lib.zm_index.restype = ctypes.c_int
    lib.zm_num_moments.restype = ctypes.c_int
    for nmax in [0, 1, 2, 3, 20, 99, 100, 200, 255, 500]:
        pl = oracle.pairs(nmax)
        assert lib.zm_num_moments(nmax) == len(pl)
        for i, (n, m) in enumerate(pl):
            assert lib.zm_index(n, m) == i
    assert lib.zm_num_moments(-1) == -1
    for n, m in [(-1, 0), (3, 2), (2, 3), (4, -2), (5, 6)]:
        assert lib.zm_index(n, m) == -1


def test_status_strings(lib):
    lib.zm_status_str.restype = ctypes.c_char_p
    for s in range(0, -6, -1):
        assert lib.zm_status_str(s).decode().startswith("ZM_")


def test_null_arguments_rejected_without_device(lib):
    lib.zm_plan_ex.restype = ctypes.c_int
    lib.zm_plan_info.restype = ctypes.c_int
    lib.zm_workspace_size.restype = ctypes.c_int
    lib.zm_destroy.restype = ctypes.c_int
    assert lib.zm_plan_ex(None, None) == -1
    assert lib.zm_plan_info(None, None) == -1
    assert lib.zm_workspace_size(None, 1, None) == -1
    assert lib.zm_destroy(None) == -1
