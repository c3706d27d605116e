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


def test_binding_structs_match_the_header(tmp_path):
    """Every structure the binding passes across the C ABI has the header's
    size and field offsets (a C program compiled against include/mcdose.h
    reports them)."""
    import subprocess

    from paper_0910_0329_amd import mcdose
    pairs = [("mcd_grid", mcdose.Grid), ("mcd_source", mcdose.Source),
             ("mcd_energy_balance", mcdose.EnergyBalance), ("mcd_opts", mcdose.Opts),
             ("mcd_result", mcdose.Result), ("mcd_batch_item", mcdose.BatchItem),
             ("mcd_serve_config", mcdose.ServeConfig), ("mcd_serve_stats", mcdose.ServeStats)]
    lines = ['#include <stdio.h>', '#include "mcdose.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append('printf("mcd_history_record size %zu\\n", sizeof(mcd_history_record));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, py in pairs:
        assert int(got[f"{cname} size"]) == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert int(got[f"{cname} {f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])
    # the history record matches its numpy view
    assert mcdose.HISTORY_DTYPE.itemsize == int(got["mcd_history_record size"])


def test_unknown_option_is_an_error():
    from paper_0910_0329_amd import mcdose
    assert mcdose.make_opts(sched_fetch_div=3).sched_fetch_div == 3
    with pytest.raises(TypeError):
        mcdose.make_opts(sched_fetch_dvi=3)
