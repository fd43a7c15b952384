"""The allocation-free matching call (hdp_match_layer_noalloc) against
hdp_match_layer on the same forests: aggregated volumes and labels must be
identical bit for bit, over consecutive calls that reuse the library's fixed
scratch array with different sizes (largest first), on the fused narrow-row
path (right image as FP32 and packed) and on the wide-row path."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1509_08197_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1509_08197_amd import hdp
    hdp.lib()
    return hdp


def _rgb(pair):
    L = torch.from_numpy(pair.left.reshape(-1, 3).copy()).cuda()
    R = torch.from_numpy(pair.right.reshape(-1, 3).copy()).cuda()
    return L, R


def _layer(H, pair, level, S=2, L=3, window=4):
    """Images, shapes and forest of one layer of the HDP step of `pair`."""
    Lr, Rr = _rgb(pair)
    shapes = [(pair.shape[0], pair.shape[1], pair.dmax)]
    res = H.hdp_stereo(Lr, Rr, shapes, S=S, L=L, window=window)
    lp, rp = H.pyramid_views(Lr, Rr, shapes, S, L)
    lv = H.level_shapes(shapes, S, L)
    return lp[level], rp[level], lv[level], res[level].forest


def _full(H, pair):
    Lr, Rr = _rgb(pair)
    shapes = [(pair.shape[0], pair.shape[1], pair.dmax)]
    lp, rp = H.pyramid_views(Lr, Rr, shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    return lp[0], rp[0], shapes, f


def _compare(H, left, right, shapes, f, what):
    print(f"noalloc case: {what}, n={f.n}, width={f.width}", flush=True)
    a_ref, d_ref = H.match_layer(left, right, shapes, f)
    # fill the outputs with garbage first: the call must write every entry it owns
    a_na = torch.full_like(a_ref, float("nan"))
    d_na = torch.full_like(d_ref, -7)
    H.match_layer_noalloc(left, right, shapes, f, agg=a_na, disp=d_na)
    torch.cuda.synchronize()
    assert torch.equal(d_na, d_ref), f"{what}: labels differ"
    # compare the valid columns of every row (padding columns are not part of the output)
    node = f.array("node").long()
    width = (f.array("hi") - f.array("lo") + 1)[node]
    cols = torch.arange(f.width, device=a_ref.device)[None, :] < width[:, None]
    assert torch.equal(a_na[cols], a_ref[cols]), f"{what}: aggregated volumes differ"
    assert f.read_info()[7] == 0, f"{what}: consistency guard tripped"


def test_noalloc_matches_workspace_call(H):
    # 1) the largest case: layer 0 of the 1344x1104 pair (HDP windows of 10 labels)
    big = scenes.workload(2)
    left, right, shapes, f = _layer(H, big, 0)
    need = H.lib().hdp_aggregate_workspace_bytes(f.n, f.width)
    assert need <= H.noalloc_max_bytes()
    _compare(H, left, right, shapes, f, "1344x1104 layer 0")
    del left, right, f
    # 2) a smaller input right after it: the 160x120 pair's layer 0 and its top layer
    small = scenes.workload(1)
    for level in (0, 2):
        left, right, shapes, f = _layer(H, small, level, L=2, window=2)
        _compare(H, left, right, shapes, f, f"160x120 layer {level}")
    # 3) 64-label rows (fused passes, right image packed in the scratch array)
    wide = scenes.small_scene(77, 48, 64, 63)
    left, right, shapes, f = _full(H, wide)
    assert f.width == 64
    _compare(H, left, right, shapes, f, "64x48 full range, 64 labels")
    # 4) wide rows (66 labels, not in fours: cost volume in the scratch array)
    wide = scenes.small_scene(78, 40, 60, 65)
    left, right, shapes, f = _full(H, wide)
    assert f.width == 66
    _compare(H, left, right, shapes, f, "60x40 full range, 66 labels")


def test_noalloc_rejects_oversize(H):
    """A layer whose scratch exceeds the fixed array is refused with
    HDP_EWORKSPACE and nothing is written."""
    pair = scenes.small_scene(5, 16, 16, 15)
    left, right, shapes, f = _full(H, pair)
    st = H.ForestStruct.from_buffer_copy(f.st)
    st.n = 6 << 20  # pretend a 6M-pixel layer: only the size is read before the refusal
    import ctypes as C
    p = H.cost_params()
    agg = torch.zeros((f.n, f.width), device="cuda")
    disp = torch.full((f.n,), -3, dtype=torch.int32, device="cuda")
    code = H.lib().hdp_match_layer_noalloc(
        H._ptr(left), H._ptr(right), H._shapes(shapes), 1, C.byref(st), int(f.width), C.byref(p),
        C.c_float(0.1), H._ptr(agg), H._ptr(disp), H._stream())
    torch.cuda.synchronize()
    assert code == -3
    assert (disp == -3).all() and (agg == 0).all()
