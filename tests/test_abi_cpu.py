"""The C ABI library loads, exports what include/tnn.h declares, and rejects
bad arguments before touching the GPU.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2112_10408_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tnn_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    declared = _declared()
    assert {"tnn_build_segments", "tnn_query"} <= declared
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert declared <= set(capi.exported_symbols())


def test_status_strings():
    L = capi.lib()
    for code in range(0, -8, -1):
        s = L.tnn_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.tnn_status_string(-99).decode() == "unknown status"


def _ws(off, seg_len):
    off = np.ascontiguousarray(off, dtype=np.int64)
    nb = ctypes.c_size_t(0)
    rc = capi.lib().tnn_build_segments_workspace(off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1,
                                                 seg_len, ctypes.byref(nb))
    return rc, nb.value


def test_build_workspace_validation():
    rc, n = _ws([0, 50, 100], 16)
    assert rc == capi.TNN_OK and n > 0
    assert _ws([0, 50, 100], 0)[0] == capi.TNN_E_ARG
    assert _ws([0, 50, 100], 65)[0] == capi.TNN_E_ARG
    assert _ws([0, 50, 40], 16)[0] == capi.TNN_E_ARG  # decreasing offsets
    assert _ws([1, 50], 16)[0] == capi.TNN_E_ARG      # must start at 0
    rc0, n0 = _ws([0], 16)                          # no trajectory at all
    assert rc0 == capi.TNN_OK
    # workspace grows with the data
    assert _ws([0, 5000], 16)[1] > _ws([0, 50], 16)[1]


def test_query_rejects_bad_arguments_without_gpu():
    L = capi.lib()
    p = capi.TnnQueryParams()
    p.scale[:] = [1, 1, 10, 0.05]
    p.k = 8
    q = capi.TnnPoints(None, None, None, None, 0)
    nb = ctypes.c_size_t(0)
    # null / unbuilt index
    assert L.tnn_query(None, q, ctypes.byref(p), None, None, None, 0, None) == capi.TNN_E_ARG
    idx = capi.TnnIndex()
    assert L.tnn_query_workspace(ctypes.byref(idx), 10, ctypes.byref(p), ctypes.byref(nb)) == capi.TNN_E_ARG
    assert L.tnn_index_info(ctypes.byref(idx), None, None, None, None) == capi.TNN_E_ARG


def test_build_rejects_bad_arguments_without_gpu():
    L = capi.lib()
    off = np.array([0, 10], dtype=np.int64)
    pts = capi.TnnPoints(None, None, None, None, 10)  # null coordinate arrays
    out = capi.TnnIndex()
    rc = L.tnn_build_segments(pts, off.ctypes.data_as(ctypes.c_void_p), 1, 16, None,
                              ctypes.c_void_p(1), 1 << 20, None, ctypes.byref(out))
    assert rc == capi.TNN_E_ARG


def _decl_arg_counts():
    out = {}
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, fn)).read(), flags=re.S)
        for m in re.finditer(r"\b(tnn_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", src):
            args = m.group(2).strip()
            out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_header_arity():
    L = capi.lib()
    counts = _decl_arg_counts()
    assert counts
    for name, n in counts.items():
        assert len(getattr(L, name).argtypes) == n, name


def test_gka_rejects_bad_arguments_without_gpu():
    L = capi.lib()
    E = capi.TNN_E_ARG
    assert L.tnn_gka_average(None, None, 10, 0, None, 2, 100, None, None) == E    # k = 0
    assert L.tnn_gka_average(None, None, 10, 65, None, 2, 100, None, None) == E   # k > 64
    assert L.tnn_gka_average(None, None, 10, 8, None, 0, 100, None, None) == E    # no component
    assert L.tnn_gka_average(None, None, 10, 8, None, 9, 100, None, None) == E    # too many
    assert L.tnn_gka_average(None, None, -1, 8, None, 2, 100, None, None) == E    # negative count
    assert L.tnn_gka_average(None, None, 10, 8, None, 2, 100, None, None) == E    # null buffers
    assert L.tnn_gka_average(None, None, 0, 8, None, 2, 100, None, None) == capi.TNN_OK  # nothing to do


def test_query_params_struct_matches_header():
    """The binding's tnn_query_params has the header's fields, in order (the
    struct crosses the C ABI by value)."""
    src = open(os.path.join(ROOT, "include", "tnn.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} tnn_query_params;", src).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\**\s*([a-z_0-9]+)\s*(?:\[[^\]]*\])?\s*;", body)
    assert names == [f[0] for f in capi.TnnQueryParams._fields_]


def test_noalloc_rejects_bad_arguments_before_the_gpu():
    """Argument checks of the scratch-free entry point run on the host,
    before any device is touched."""
    L = capi.lib()
    pts = capi.TnnPoints(None, None, None, None, 0)
    assert L.tnn_query_noalloc(None, pts, None, None, None, None) == capi.TNN_E_ARG
    idx = capi.TnnIndex()
    p = capi.TnnQueryParams()
    p.scale[:] = [1.0, 1.0, 10.0, 0.05]
    p.k = 8
    # an index that was never built
    assert L.tnn_query_noalloc(ctypes.byref(idx), pts, ctypes.byref(p), None, None, None) == capi.TNN_E_ARG
