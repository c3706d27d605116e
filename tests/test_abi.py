"""The C ABI library loads and exports every function that include/*.h declares
(no device calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(mcd_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mcd_create", "mcd_load_materials", "mcd_load_phantom", "mcd_simulate"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_0910_0329_amd import mcdose
    if not os.path.exists(mcdose.LIB_PATH):
        pytest.fail("libmcdose.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(mcdose.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    assert set(mcdose.EXPORTED) <= set(declared_functions())


def test_status_strings_without_device():
    from paper_0910_0329_amd import mcdose
    L = mcdose.lib()
    assert L.mcd_status_string(0) == b"ok"
    assert b"overflow" in L.mcd_status_string(-4)
    assert L.mcd_last_error(None) == b"null context"
