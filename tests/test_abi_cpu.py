"""Host-only checks of the C ABI: the library loads, exports every function
include/annkin.h declares, and rejects bad arguments before touching a GPU."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "annkin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ak_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_08483_amd import annkin
    return annkin.lib()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("ak_load_mechanism", "ak_eval_source", "ak_free_mechanism",
                     "ak_last_error", "ak_error_count"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu(lib):
    from paper_2008_08483_amd import annkin
    out = C.c_void_p()
    assert lib.ak_load_mechanism(None, 0, C.byref(out)) == -1
    assert b"null" in lib.ak_last_error()
    d = annkin.MechanismDesc()
    d.n_species = 0
    assert lib.ak_load_mechanism(C.byref(d), 0, C.byref(out)) == -1
    d.n_species, d.n_reactions = 257, 1          # species indices are bytes
    assert lib.ak_load_mechanism(C.byref(d), 0, C.byref(out)) == -7
    assert b"257 species" in lib.ak_last_error()
    assert lib.ak_eval_source(None, 0, None, None, None, 0, 0, None, 0, None) == -1
    assert lib.ak_free_mechanism(None) == 0
    assert lib.ak_mechanism_n_species(None) == -1
    assert lib.ak_version().startswith(b"annkin")
