"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments on the host (before any GPU work)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdp.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1509_08197_amd import hdp
    if not os.path.exists(hdp.LIB_PATH):
        from paper_1509_08197_amd import build
        build.build(verbose=False)
    return hdp


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"HDP_API\s+[\w\s\*]+?\b(hdp_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    L = C.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_level_shapes_match_oracle(lib, orc):
    for H, W, d, L in [(1104, 1344, 255, 3), (375, 1242, 191, 2), (1, 1, 0, 4), (7, 3, 9, 3)]:
        got = lib.level_shapes([(H, W, d)], 2, L)
        Hs, Ws, ds = orc.level_dims(H, W, d, 2, L)
        assert [s[0] for s in got] == [(h, w, dd) for h, w, dd in zip(Hs, Ws, ds)]


def test_status_strings(lib):
    L = lib.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.hdp_status_str(code)


def _fake_forest(lib, n):
    """Bind a forest to a host buffer: pointers only, nothing is dereferenced."""
    L = lib.lib()
    nbytes = L.hdp_forest_bytes(n)
    buf = np.zeros(nbytes + 512, np.uint8)
    addr = (buf.ctypes.data + 255) & ~255
    st = lib.ForestStruct()
    assert L.hdp_forest_bind(C.c_void_p(addr), nbytes, n, C.byref(st)) == 0
    return buf, st, addr


def test_forest_bind_errors(lib):
    L = lib.lib()
    n = 100
    nbytes = L.hdp_forest_bytes(n)
    buf = np.zeros(nbytes + 512, np.uint8)
    addr = (buf.ctypes.data + 255) & ~255
    st = lib.ForestStruct()
    assert L.hdp_forest_bind(C.c_void_p(addr + 4), nbytes, n, C.byref(st)) == -1  # unaligned
    assert L.hdp_forest_bind(C.c_void_p(addr), nbytes - 1, n, C.byref(st)) == -3  # too small
    assert L.hdp_forest_bind(None, nbytes, n, C.byref(st)) == -1


def test_build_tree_validation(lib):
    L = lib.lib()
    H, W = 8, 8
    shapes = lib._shapes([(H, W, 63)])
    buf, st, addr = _fake_forest(lib, H * W)
    dummy = C.c_void_p(addr)  # never dereferenced: every call below fails validation
    ws = L.hdp_build_tree_workspace_bytes(H * W)
    # null image
    assert L.hdp_build_tree(None, shapes, 1, 0, None, None, 0, 19, 20, 64, C.byref(st),
                            dummy, ws, None) == -1
    # empty batch
    assert L.hdp_build_tree(dummy, shapes, 0, 0, None, None, 0, 19, 20, 64, C.byref(st),
                            dummy, ws, None) == -2
    # (outside the exact regime, width 10 with beta 3/5, the call runs the
    # sequential process on the device: not callable here)
    # the row width must hold a tree's interval: at
    # least max_width
    assert L.hdp_build_tree(dummy, shapes, 1, 0, dummy, dummy, 10, 3, 5, 9, C.byref(st),
                            dummy, ws, None) == -1
    # workspace too small
    assert L.hdp_build_tree(dummy, shapes, 1, 0, dummy, dummy, 10, 19, 20, 10, C.byref(st),
                            dummy, ws - 1, None) == -3
    # full range needs width >= dmax + 1
    assert L.hdp_build_tree(dummy, shapes, 1, 0, None, None, 0, 19, 20, 32, C.byref(st),
                            dummy, ws, None) == -1
    # forest bound for a different size
    shapes2 = lib._shapes([(H, W + 1, 63)])
    assert L.hdp_build_tree(dummy, shapes2, 1, 0, None, None, 0, 19, 20, 64, C.byref(st),
                            dummy, ws, None) == -1


def test_shape_validation(lib):
    L = lib.lib()
    dummy = C.c_void_p(256)
    bad = [(0, 5, 3), (5, 0, 3), (5, 5, -1), (5, 5, 256), (3000, 3000, 10)]
    for s in bad:
        assert L.hdp_pyramid(dummy, lib._shapes([s]), 1, 2, 1, dummy, None) == -2, s
    many = [(4, 4, 3)] * 65
    assert L.hdp_pyramid(dummy, lib._shapes(many), 65, 2, 1, dummy, None) == -2
    assert L.hdp_pyramid(dummy, lib._shapes([(4, 4, 3)]), 1, 3, 1, dummy, None) == -1  # S != 2


def test_predict_range_shape_mismatch(lib):
    L = lib.lib()
    dummy = C.c_void_p(256)
    up = lib._shapes([(4, 4, 7)])
    low_ok = lib._shapes([(8, 8, 15)])
    low_bad = lib._shapes([(9, 8, 15)])
    assert L.hdp_predict_range(dummy, up, low_bad, 1, 2, 4, dummy, dummy, None) == -2
    assert L.hdp_predict_range(None, up, low_ok, 1, 2, 4, dummy, dummy, None) == -1


def test_aggregate_validation(lib):
    L = lib.lib()
    n = 64
    buf, st, addr = _fake_forest(lib, n)
    dummy = C.c_void_p(addr)
    ws = L.hdp_aggregate_workspace_bytes(n, 16)
    assert L.hdp_aggregate(C.byref(st), 16, dummy, C.c_float(0.0), dummy, None, dummy, ws,
                           None) == -1  # sigma must be > 0
    assert L.hdp_aggregate(C.byref(st), 16, dummy, C.c_float(0.1), dummy, None, dummy, ws - 1,
                           None) == -3
    assert L.hdp_aggregate(C.byref(st), 300, dummy, C.c_float(0.1), dummy, None, dummy, ws,
                           None) == -1  # width > 256


def test_match_layer_validation(lib):
    """hdp_match_layer rejects bad arguments on the host, before any launch."""
    L = lib.lib()
    H, W = 8, 8
    n = H * W
    buf, st, addr = _fake_forest(lib, n)
    dummy = C.c_void_p(addr)
    shapes = (lib.Shape * 1)(lib.Shape(H, W, 15))
    p = lib.cost_params()
    ws = L.hdp_aggregate_workspace_bytes(n, 10)
    ok = dict(left=dummy, right=dummy, shapes=shapes, n_pairs=1, f=C.byref(st), width=10,
              p=C.byref(p), sigma=C.c_float(0.1), agg=dummy, disp=dummy, ws=dummy, wsb=ws)

    def call(**kw):
        a = dict(ok, **kw)
        return L.hdp_match_layer(a["left"], a["right"], a["shapes"], a["n_pairs"], a["f"],
                                 a["width"], a["p"], a["sigma"], a["agg"], a["disp"], a["ws"],
                                 a["wsb"], None)

    assert call(left=None) == -1
    assert call(disp=None) == -1
    assert call(sigma=C.c_float(0.0)) == -1
    assert call(width=300) == -1
    assert call(wsb=ws - 1) == -3
    other = (lib.Shape * 1)(lib.Shape(H, W + 1, 15))  # forest does not match the batch
    assert call(shapes=other) == -1
    assert call(n_pairs=0) == -2
    bad = lib.cost_params(border=2)  # border policy is 0 or 1
    assert call(p=C.byref(bad)) == -1
    assert L.hdp_cost_volume(dummy, dummy, shapes, 1, C.byref(st), 10, C.byref(bad), dummy,
                             None) == -1


def test_workspace_sizes_grow(lib):
    L = lib.lib()
    a = [L.hdp_build_tree_workspace_bytes(n) for n in (10, 1000, 100000)]
    b = [L.hdp_aggregate_workspace_bytes(n, 10) for n in (10, 1000, 100000)]
    assert a == sorted(a) and b == sorted(b)
    assert L.hdp_aggregate_workspace_bytes(1000, 256) > L.hdp_aggregate_workspace_bytes(1000, 10)


def test_match_layer_noalloc_rejects_oversize(lib):
    """The allocation-free matching call refuses, before any HIP call, a layer
    whose scratch space exceeds its fixed array."""
    L = lib.lib()
    cap = lib.noalloc_max_bytes()
    assert cap == 256 << 20
    # a layer of 4M pixels at 32 labels per row needs more than the array holds;
    # only the forest's size is read before the refusal
    st = lib.ForestStruct()
    st.n = 4 << 20
    assert L.hdp_aggregate_workspace_bytes(st.n, 32) > cap
    shapes = (lib.Shape * 1)(lib.Shape(2048, 2048, 255))
    p = lib.cost_params()
    d = C.c_void_p(256)
    assert L.hdp_match_layer_noalloc(d, d, shapes, 1, C.byref(st), 32, C.byref(p),
                                     C.c_float(0.1), d, d, None) == -3
    assert L.hdp_match_layer_noalloc(d, d, shapes, 1, None, 32, C.byref(p), C.c_float(0.1), d,
                                     d, None) == -1
    assert L.hdp_match_layer_noalloc(d, d, shapes, 1, C.byref(st), 300, C.byref(p),
                                     C.c_float(0.1), d, d, None) == -1
    # the single-pair 1344x1104 layer 0 at 10 labels per row fits
    assert L.hdp_aggregate_workspace_bytes(1344 * 1104, 10) <= cap
