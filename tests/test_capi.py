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


def test_binding_declares_argument_types():
    """Every entry point with arguments has ctypes argument types, so that
    pointers and 64-bit sizes are never passed as C int."""
    lib = graphlet4.load()
    for name in graphlet4.EXPORTS:
        if name == "gc_last_error":
            continue
        assert getattr(lib, name).argtypes is not None, name


def test_error_strings_without_device():
    lib = graphlet4.load()
    assert lib.gc_strerror(0) == b"ok"
    assert lib.gc_strerror(-1) == b"invalid argument"
    o = graphlet4.Options()
    assert lib.gc_options_default(ctypes.byref(o)) == 0
    assert o.radius == 2 and abs(o.slack - 0.25) < 1e-6
    assert lib.gc_options_default(None) == -1
    assert lib.gc_copy_tuning(None, None) == -1


def test_server_admission_refusal_without_device():
    """A fake memory budget refuses a graph before any device work."""
    from paper_2308_14493_amd.graphlet4 import Server, GraphletError
    with Server(hbm_budget_bytes=1024, hbm_reserve_bytes=0) as srv:
        try:
            srv.add_graph(100, [0, 1], [1, 2])
        except GraphletError as e:
            assert e.code == -2 and "HBM" in str(e)
        else:
            raise AssertionError("admission should refuse")
    lib = graphlet4.load()
    o = graphlet4.ServerOpts()
    lib.gc_server_opts_default(ctypes.byref(o))
    o.max_graphs = 0
    h = ctypes.c_void_p()
    assert lib.gc_server_create(ctypes.byref(o), ctypes.byref(h)) == -1


def test_footprint_estimate_without_device():
    """The admission estimate is host arithmetic: positive, growing with the
    graph, and it rejects ids outside [0, n)."""
    from paper_2308_14493_amd.graphlet4 import footprint, GraphletError
    small = footprint(100, [0, 1], [1, 2])
    big = footprint(100000, list(range(0, 99999)), list(range(1, 100000)))
    assert 0 < small < big
    try:
        footprint(10, [0], [10])
    except GraphletError as e:
        assert e.code == -1
    else:
        raise AssertionError("an id outside [0, n) must be rejected")


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of gc_options, gc_batch_stats, gc_batch_desc and
    gc_server_opts have the C layout: every field at the offset the header
    gives it, and the same total size (compiled here with gcc)."""
    import subprocess
    mirrors = {"gc_options": graphlet4.Options, "gc_batch_stats": graphlet4.BatchStats,
               "gc_batch_desc": graphlet4.BatchDesc, "gc_server_opts": graphlet4.ServerOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "graphlet4.h"', 'int main(void) {']
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ['return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
