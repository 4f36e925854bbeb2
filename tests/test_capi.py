"""Host-side checks of the C ABI library (no GPU needed): it loads and
exports every function that include/graphlet4.h declares."""
import ctypes
import os
import re

from paper_2308_14493_amd import graphlet4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "graphlet4.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert sorted(graphlet4.EXPORTS) == declared_functions()


def test_library_exports_every_symbol():
    lib = graphlet4.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_error_strings_without_device():
    lib = graphlet4.load()
    assert lib.gc_strerror(0) == b"ok"
    assert lib.gc_strerror(-1) == b"invalid argument"
    o = graphlet4.Options()
    assert lib.gc_options_default(ctypes.byref(o)) == 0
    assert o.radius == 2 and abs(o.slack - 0.25) < 1e-6
    assert lib.gc_options_default(None) == -1
