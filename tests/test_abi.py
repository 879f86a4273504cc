"""The C-ABI library loads and exports every entry point include/sg.h declares
(CPU only: argument checks and workspace sizing, no kernel launches)."""
import ctypes as C
import os
import re

import pytest

import paper_2605_10135_amd as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sg.lib()
    names = declared()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name
    # the binding declares the same set
    assert set(sg.exported_symbols()) == set(names)


def test_status_strings_and_version():
    L = sg.lib()
    assert L.sg_status_str(0) == b"SG_OK"
    assert b"invalid argument" in L.sg_status_str(-1)
    assert b"gfx950" in L.sg_version()


def test_argument_errors_are_reported_without_launching():
    L = sg.lib()
    # k = 0 is rejected on the host before anything touches a device
    rc = L.sg_knn_graph(C.c_void_p(1), 0, 10, 8, 8, 0, 0, 0, 0, C.c_void_p(1), None, None, None, 0, None)
    assert rc == -1
    assert b"k must be" in L.sg_last_error()
    rc = L.sg_prune(C.c_void_p(1), 10, 8, 9, None, C.c_void_p(1), None, 0, None)
    assert rc == -1
    assert b"R must be" in L.sg_last_error()
    # too-small workspace
    rc = L.sg_prune(C.c_void_p(1), 10, 8, 4, None, C.c_void_p(1), None, 0, None)
    assert rc == -3
    off = (C.c_int64 * 3)(0, 5, 4)
    rc = L.sg_merge(2, off, C.c_void_p(1), C.c_void_p(1), 4, 10, 8, C.c_void_p(1), C.c_void_p(1), None,
                    0, None)
    assert rc == -1
    assert b"non-decreasing" in L.sg_last_error()
    rc = L.sg_search(C.c_void_p(1), 0, 10, 8, 8, 0, C.c_void_p(1), 4, C.c_void_p(1), 3, 8, 10, 5, -1,
                     C.c_void_p(1), None, None, 0, None)
    assert rc == -1


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_workspace_sizes(prec):
    L = sg.lib()
    out = C.c_size_t(0)
    assert L.sg_knn_graph_workspace_size(1000, 96, 32, prec, 0, C.byref(out)) == 0
    assert out.value > 1000 * 32 * 8
    assert L.sg_prune_workspace_size(1000, 64, 32, C.byref(out)) == 0
    assert out.value >= 1000 * 32 * 8 + 1000 * 24      # P and 32-bit reverse keys, three counters per row
    off = (C.c_int64 * 3)(0, 600, 1100)
    assert L.sg_merge_workspace_size(2, off, 800, C.byref(out)) == 0
    assert out.value >= 1100 * 16
    assert L.sg_partition_workspace_size(1000, 16, 4, 2, C.byref(out)) == 0
    assert L.sg_search_workspace_size(1000, 16, 50, C.byref(out)) == 0
