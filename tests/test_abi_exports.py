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
