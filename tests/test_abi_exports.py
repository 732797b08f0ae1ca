"""The C-ABI library loads on a CPU-only host and exports every entry point
that include/amg.h declares; the binding refuses to run without it."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:amg_status|void|const char\*)\s+(amg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2602_05686_amd as amg
    from paper_2602_05686_amd import build

    if not os.path.exists(amg.LIB_PATH):
        build.build()
    return amg.load()


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for required in ("amg_setup", "amg_pcg_solve", "amg_vcycle", "amg_free", "amg_hierarchy_info",
                     "amg_get_aggregates", "amg_get_soc_mask", "amg_options_default"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2602_05686_amd as amg

    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in amg.h but not exported"
    assert set(declared_functions()) == set(amg.EXPORTED)


def test_host_only_calls(lib):
    import paper_2602_05686_amd as amg

    o = amg.options(dim=2)
    assert o.theta == 0.08 and o.max_coarse == 5000 and o.max_levels == 10 and o.cheb_degree == 2
    assert lib.amg_status_string(0) == b"ok"
    assert lib.amg_status_string(5) == b"coarsening stagnated"
    # argument validation happens before any device work
    h = ctypes.c_void_p()
    code = lib.amg_setup(0, None, None, None, 0, 0, None, None, None, ctypes.byref(o), 0, None, ctypes.byref(h))
    assert code == 1 and h.value is None
    assert b"n must" in lib.amg_last_error()


def test_missing_library_fails_loudly(monkeypatch):
    import paper_2602_05686_amd._lib as L

    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", os.path.join(ROOT, "no_such_library.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.load()


def test_ctypes_structs_match_the_header(tmp_path):
    """Field offsets and sizes of the binding's structs equal the C layout."""
    import shutil
    import subprocess

    from paper_2602_05686_amd import _lib

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {
        "amg_options": _lib.Options, "amg_solve_info": _lib.SolveInfo, "amg_hierarchy_stats": _lib.HierStats,
        "amg_server_stats": _lib.ServerStats, "amg_request_stats": _lib.RequestStats,
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "amg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_server_argument_checks_precede_device_work(lib):
    import paper_2602_05686_amd as amg

    o = amg.options(dim=3)
    s = ctypes.c_void_p()
    assert lib.amg_server_create(ctypes.byref(o), 0, 4, 1, ctypes.byref(s)) == 1 and s.value is None
    assert b"budget" in lib.amg_last_error()
    assert lib.amg_server_create(ctypes.byref(o), 1 << 30, 0, 1, ctypes.byref(s)) == 1
    assert lib.amg_server_create(ctypes.byref(o), 1 << 30, 4, 0, ctypes.byref(s)) == 1
    nd = ctypes.c_int32()
    assert lib.amg_server_poll(None, 0.0, None, 0, ctypes.byref(nd)) == 1
    lib.amg_server_set_batch_wait.argtypes = [ctypes.c_void_p, ctypes.c_double]
    assert lib.amg_server_set_batch_wait(None, 0.5) == 1
    lib.amg_server_destroy(None)
