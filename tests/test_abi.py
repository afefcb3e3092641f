"""CPU checks of the C-ABI library: it loads, exports every symbol include/topktri.h declares,
and rejects bad arguments before touching the device."""
import ctypes
import math
import os
import re

import pytest

import paper_1910_00692_amd as tt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "topktri.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tt.LIB_PATH):
        tt.build()
    return tt.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("graph_load", "topk_triangles", "sample_heavy_triangles", "graph_free", "tt_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tt.EXPORTED)


def test_struct_sizes():
    assert ctypes.sizeof(tt.Triangle) == 24
    text = open(HEADER).read()
    assert "uint32_t i, j, l, _pad;" in text


def test_argument_errors_before_device_work(lib):
    h = ctypes.c_void_p()
    assert lib.graph_load(3, 2, None, None, None, ctypes.byref(h)) == tt.TT_E_ARG
    assert b"NULL" in lib.tt_last_error()
    assert lib.graph_load(3, 0, None, None, None, None) == tt.TT_E_ARG
    one = (ctypes.c_uint32 * 1)(0)
    assert lib.graph_load(3, 2**32, one, one, one, ctypes.byref(h)) == tt.TT_E_TOO_LARGE
    n_out = ctypes.c_uint32(7)
    out = (tt.Triangle * 4)()
    assert lib.topk_triangles(None, 4, 1.0, out, ctypes.byref(n_out)) == tt.TT_E_ARG
    assert n_out.value == 0
    assert lib.sample_heavy_triangles(None, 4, 1.0, 10, 1, out, ctypes.byref(n_out)) == tt.TT_E_ARG
    assert lib.sample_heavy_triangles_ex(None, 4, 1.0, 10, 1, math.nan, None, out, ctypes.byref(n_out),
                                         None) == tt.TT_E_ARG
    lib.graph_free(None)  # NULL-safe
    assert lib.graph_num_edges(None) == 0 and lib.graph_num_vertices(None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(tt, "_lib", None)
    monkeypatch.setattr(tt, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(tt.LibraryMissing):
        tt.library()


def test_server_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.server_create(None, 4, 1 << 30, ctypes.byref(h)) == tt.TT_E_ARG
    assert lib.server_create(None, 4, 1 << 30, None) == tt.TT_E_ARG
    t = ctypes.c_uint64(5)
    assert lib.server_submit(None, 10, 1.0, None, 0, ctypes.byref(t)) == tt.TT_E_ARG
    n_out = ctypes.c_uint32(3)
    assert lib.server_wait(None, 1, None, ctypes.byref(n_out), None) == tt.TT_E_ARG and n_out.value == 0
    assert lib.server_info(None, None, None, None, None, None) == tt.TT_E_ARG
    assert lib.server_request_bytes(None, 10, 0) == 0
    lib.server_destroy(None)  # NULL-safe


def test_batch_argument_errors(lib):
    h = ctypes.c_void_p()
    n = (ctypes.c_uint32 * 1)(3)
    m = (ctypes.c_uint64 * 1)(2)
    assert lib.batch_load(1, n, m, None, None, None, ctypes.byref(h)) == tt.TT_E_ARG
    assert lib.batch_load(1, None, m, None, None, None, ctypes.byref(h)) == tt.TT_E_ARG
    assert lib.batch_load(0, None, None, None, None, None, None) == tt.TT_E_ARG
    big = (ctypes.c_uint32 * 2)(2**31, 2**31)
    zero = (ctypes.c_uint64 * 2)(0, 0)
    assert lib.batch_load(2, big, zero, None, None, None, ctypes.byref(h)) == tt.TT_E_TOO_LARGE
    n_out = (ctypes.c_uint32 * 2)(5, 5)
    assert lib.batch_topk(None, 10, 1.0, None, n_out) == tt.TT_E_ARG
    assert lib.batch_topk_ex(None, 10, 1.0, -1, 0, None, n_out, None) == tt.TT_E_ARG
    assert lib.batch_num_graphs(None) == 0 and lib.batch_num_configs() >= 2
    lib.batch_free(None)  # NULL-safe


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's size and field offsets."""
    import subprocess
    mirrors = {"tt_triangle": tt.Triangle, "tt_query_stats": tt.QueryStats, "tt_batch_stats": tt.BatchStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "topktri.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
