"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times: trees and level order bit-exact on whole arrays, aggregated costs on
sampled label slices the oracle computes one by one, WTA labels identical
except at near-ties.  Batched runs are checked on spot pairs against
single-pair oracle runs."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1509_08197_amd import scenes

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1509_08197_amd import hdp
    hdp.lib()
    return hdp


def rgb_dev(*imgs):
    return torch.from_numpy(np.ascontiguousarray(
        np.concatenate([im.reshape(-1, 3) for im in imgs]))).cuda()


def rows_to_pixels(vol, node, lo, hi, labels, n):
    """Values of a [n][width] volume at the given labels, pixel order (NaN outside)."""
    out = np.full((len(labels), n), np.nan)
    for k, x in enumerate(labels):
        j = x - lo[node]
        ok = (j >= 0) & (x <= hi[node]) & (j < vol.shape[1])
        out[k, node[ok]] = vol[ok, j[ok]]
    return out


def assert_rel(got, ref, what):
    m = ~np.isnan(ref)
    assert np.array_equal(np.isnan(got), np.isnan(ref)), f"{what}: support differs"
    err = np.abs(got[m] - ref[m]) / np.abs(ref[m])
    assert err.max() <= REL, f"{what}: max rel err {err.max():.3g}"


def check_layer(H, orc, lres, ores, labels, what):
    f = lres.forest
    n = f.n
    torch.cuda.synchronize()
    A = {k: f.array(k).cpu().numpy() for k in ("parent", "depth", "order", "node", "lo", "hi",
                                                 "level_ptr")}
    info = f.read_info()
    assert info[7] == 0, f"{what}: guard {info[7]}"
    np.testing.assert_array_equal(A["parent"], ores["parent"], err_msg=f"{what} parent")
    np.testing.assert_array_equal(A["depth"], ores["depth"], err_msg=f"{what} depth")
    np.testing.assert_array_equal(A["order"], ores["order"], err_msg=f"{what} order")
    nl = ores["n_levels"]
    np.testing.assert_array_equal(A["level_ptr"][:nl + 1], ores["level_ptr"])
    got = rows_to_pixels(lres.agg.cpu().numpy(), A["node"], A["lo"], A["hi"], labels, n)
    assert_rel(got, ores["sample_agg"], f"{what} aggregate")
    d = lres.disp.cpu().numpy()
    o = ores["disp"].ravel()
    mism = d != o
    near = (ores["c2"] - ores["c1"]) <= REL * np.abs(ores["c1"])
    assert np.all(near[mism]), f"{what}: {int((mism & ~near).sum())} WTA mismatches off near-ties"
    return int(mism.sum())


def test_full_range_1344x1104(H, orc):
    pair = scenes.workload(2)
    Hh, Ww = pair.shape
    shapes = [(Hh, Ww, 255)]
    res = H.full_range(rgb_dev(pair.left), rgb_dev(pair.right), shapes, keep=True)
    labels = [0, 37, 128, 255]
    o = orc.stereo_level(pair.left.astype(np.float64), pair.right.astype(np.float64), 255, 0,
                         sample_d=labels)
    nm = check_layer(H, orc, res, o, labels, "full range 1344x1104")
    print(f"full range: {nm} WTA near-tie mismatches")


def test_hdp_layers_1344x1104_teacher_forced(H, orc):
    """Every layer of the HDP step at full size, fed the oracle's labels of the
    layer above (no inputs from the GPU path reach the oracle)."""
    pair = scenes.workload(2)
    Hh, Ww = pair.shape
    P = scenes.HDP_PARAMS[2]
    S, L, w = P["S"], P["L"], P["window"]
    lv = H.level_shapes([(Hh, Ww, 255)], S, L)
    lp = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, 255)], S, L)
    rp = H.pyramid(rgb_dev(pair.right), [(Hh, Ww, 255)], S, L)
    ol = orc.pyramid(pair.left, S, L)
    orr = orc.pyramid(pair.right, S, L)
    # top layer: MST over the full range
    dL = lv[L][0][2]
    labels = [0, dL // 2, dL]
    o = orc.stereo_level(ol[L], orr[L], dL, L, sample_d=labels)
    r = H.stereo_level(lp[L], rp[L], lv[L], L, keep=True)
    check_layer(H, orc, r, o, labels, f"layer {L}")
    up = o["disp"]
    for l in range(L - 1, -1, -1):
        dl = lv[l][0][2]
        lo, hi = orc.predict_range(up, lv[l][0][0], lv[l][0][1], S, w, dl)
        labels = [int(np.median(lo)), int(np.median(hi)), dl]
        o = orc.stereo_level(ol[l], orr[l], dl, l, lo, hi, beta=P["beta"], sample_d=labels)
        glo, ghi = H.predict_range(torch.from_numpy(up.ravel().astype(np.int32)).cuda(),
                                   lv[l + 1], lv[l], S, w)
        np.testing.assert_array_equal(glo.cpu().numpy(), lo.ravel())
        np.testing.assert_array_equal(ghi.cpu().numpy(), hi.ravel())
        r = H.stereo_level(lp[l], rp[l], lv[l], l, glo, ghi, max_width=min(S + 2 * w, dl + 1),
                           beta=P["beta"], keep=True)
        nm = check_layer(H, orc, r, o, labels, f"layer {l}")
        np.testing.assert_array_equal(r.forest.array("lo").cpu().numpy(), o["tree_lo"])
        print(f"layer {l}: {nm} WTA near-tie mismatches")
        up = o["disp"]


def test_fused_hdp_step_1344x1104(H):
    """The HDP step as benchmarked (fused matching on every layer) against the
    three separate steps (validated against the oracle above) on the same
    forests: aggregated volumes and labels bit for bit."""
    pair = scenes.workload(2)
    Hh, Ww = pair.shape
    P = scenes.HDP_PARAMS[2]
    S, L = P["S"], P["L"]
    shapes = [(Hh, Ww, 255)]
    Lr, Rr = rgb_dev(pair.left), rgb_dev(pair.right)
    res = H.hdp_stereo(Lr, Rr, shapes, S=S, L=L, window=P["window"], beta=P["beta"])
    lv = H.level_shapes(shapes, S, L)
    lp, rp = H.pyramid_views(Lr, Rr, shapes, S, L)
    for l in range(L, -1, -1):
        f = res[l].forest
        cost = H.cost_volume(lp[l], rp[l], lv[l], f)
        agg3 = H.aggregate(f, cost, 0.1)
        disp3 = H.wta(agg3, lv[l], f)
        aggf, dispf = H.match_layer(lp[l], rp[l], lv[l], f)
        torch.cuda.synchronize()
        assert torch.equal(aggf, agg3), f"layer {l}: aggregated volumes differ"
        assert torch.equal(dispf, disp3), f"layer {l}: labels differ"
        assert torch.equal(res[l].disp, disp3), f"layer {l}: step labels differ"


def test_fused_full_range_1344x1104(H):
    """The full-range step as benchmarked (fused matching on 256-label rows:
    the cost in the up pass with the right image packed, the winner-takes-all
    in the down pass, the built-in schedule) against the three separate steps
    (validated against the oracle above) on the same forest: aggregated volume
    and labels bit for bit, the step's own labels, and a second run."""
    pair = scenes.workload(2)
    Hh, Ww = pair.shape
    shapes = [(Hh, Ww, 255)]
    Lr, Rr = rgb_dev(pair.left), rgb_dev(pair.right)
    step = H.full_range(Lr, Rr, shapes)
    lp, rp = H.pyramid_views(Lr, Rr, shapes, 2, 0)
    f = step.forest
    assert f.width == 256
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    agg3 = H.aggregate(f, cost, 0.1)
    del cost
    disp3 = H.wta(agg3, shapes, f)
    aggf, dispf = H.match_layer(lp[0], rp[0], shapes, f)
    torch.cuda.synchronize()
    assert f.read_info()[7] == 0
    assert torch.equal(aggf, agg3), "aggregated volumes differ"
    assert torch.equal(dispf, disp3), "labels differ"
    assert torch.equal(step.disp, disp3), "step labels differ"
    # a second run (the tiles of the long chains find other finished
    # predecessors from run to run) gives the same bits
    agg2, disp2 = H.match_layer(lp[0], rp[0], shapes, f)
    torch.cuda.synchronize()
    assert torch.equal(agg2, aggf) and torch.equal(disp2, dispf), "runs differ"


def tree_roots(parent):
    n = len(parent)
    root = np.where(parent >= 0, parent, np.arange(n))
    while True:
        nxt = root[root]
        if np.array_equal(nxt, root):
            return root
        root = nxt


def tree_signature(parent):
    """Per pixel: (root, size, sum of member ids, sum of parent ids) of its tree."""
    n = len(parent)
    root = tree_roots(parent)
    size = np.bincount(root, minlength=n)
    ids = np.bincount(root, weights=np.arange(n, dtype=np.float64), minlength=n)
    pars = np.bincount(root, weights=parent.astype(np.float64), minlength=n)
    return np.stack([root, size[root], ids[root], pars[root]], axis=1)


def traced_compare(layers, ores, L, S, what):
    """Compare a GPU run of the whole loop with the oracle's, layer by layer from the
    top.  layers[l] = dict(disp, parent, pix_lo, pix_hi) of the GPU, pixel order.
    Every difference must trace back to an oracle near-tie:
      * top layer: same inputs, so the same tree; a label may differ only where
        the oracle's two best aggregated costs are within REL;
      * layer l < L: a pixel interval may differ only below a pixel of layer l+1
        whose label differed; a pixel's disparity tree may differ only if its GPU
        or its oracle tree holds such a pixel; a label may differ only at an
        oracle near-tie or where the pixel's interval or tree differed.
    Returns per layer (label differences, pixels with a different tree)."""
    out = []
    up_mism = None
    for l in range(L, -1, -1):
        g, o = layers[l], ores[l]
        od = o["disp"]
        Hl, Wl = od.shape
        odisp = od.ravel()
        gap = (o["c2"] - o["c1"]) / o["c1"]
        mism = g["disp"] != odisp
        if l == L:
            np.testing.assert_array_equal(g["parent"], o["parent"], err_msg=f"{what}: top tree")
            moved = np.zeros_like(mism)
        else:
            iv = (g["pix_lo"] != o["pix_lo"].ravel()) | (g["pix_hi"] != o["pix_hi"].ravel())
            yy, xx = np.divmod(np.arange(Hl * Wl), Wl)
            Wu = layers[l + 1]["Wl"]
            above = (yy // S) * Wu + (xx // S)
            assert np.all(up_mism[above[iv]]), \
                f"{what} layer {l}: {int((iv & ~up_mism[above]).sum())} intervals differ below an equal label"
            gr, orr = tree_roots(g["parent"]), tree_roots(o["parent"])
            g_taint = np.zeros(len(gr), bool); g_taint[gr[iv]] = True
            o_taint = np.zeros(len(orr), bool); o_taint[orr[iv]] = True
            tdiff = np.any(tree_signature(g["parent"]) != tree_signature(o["parent"]), axis=1)
            ok_tree = g_taint[gr] | o_taint[orr]
            assert np.all(ok_tree[tdiff]), \
                f"{what} layer {l}: {int((tdiff & ~ok_tree).sum())} trees differ with no upstream cause"
            moved = iv | tdiff
        bad = mism & ~moved & ~(gap <= REL)
        assert not bad.any(), f"{what} layer {l}: {int(bad.sum())} label differences off near-ties"
        out.append((l, int(mism.sum()), int(moved.sum())))
        up_mism = mism
    return out


def _gpu_layers(gpu_res, off, i, lv, L):
    layers = {}
    for l in range(L, -1, -1):
        Hl, Wl, _ = lv[l][i]
        o0, n_l = off[l][i], Hl * Wl
        par = gpu_res[l].forest.array("parent").cpu().numpy()[o0:o0 + n_l]
        d = dict(disp=gpu_res[l].disp.cpu().numpy()[o0:o0 + n_l],
                 parent=np.where(par >= 0, par - o0, -1), Wl=Wl)
        if l < L:
            d["pix_lo"] = gpu_res[l].pix_lo.cpu().numpy()[o0:o0 + n_l]
            d["pix_hi"] = gpu_res[l].pix_hi.cpu().numpy()[o0:o0 + n_l]
        layers[l] = d
    return layers


@pytest.mark.batch_inputs(3, 5)
@pytest.mark.parametrize("cfg", [3, 5])
def test_batched_spot_pairs(H, orc, cfg):
    """Full batch of uneven pairs in one call (as benchmarked); spot pairs
    against single-pair oracle runs of the whole loop, every difference traced
    back to an oracle near-tie."""
    P = scenes.HDP_PARAMS[cfg]
    pairs = scenes.workload_batch(cfg)
    shapes = [(p.shape[0], p.shape[1], p.dmax) for p in pairs]
    res = H.hdp_stereo(rgb_dev(*[p.left for p in pairs]), rgb_dev(*[p.right for p in pairs]),
                       shapes, S=P["S"], L=P["L"], window=P["window"], beta=P["beta"])
    lv = H.level_shapes(shapes, P["S"], P["L"])
    off = [np.concatenate([[0], np.cumsum([h * w for h, w, _ in lv[l]])]) for l in range(P["L"] + 1)]
    for i in (0, len(pairs) // 2, len(pairs) - 1):
        pair = pairs[i]
        ores = orc.hdp_stereo(pair.left, pair.right, pair.dmax, S=P["S"], L=P["L"],
                              window=P["window"], beta=P["beta"], want_forest=True)
        stats = traced_compare(_gpu_layers(res, off, i, lv, P["L"]), ores, P["L"], P["S"],
                               f"cfg {cfg} pair {i}")
        for l, nm, nmoved in stats:
            print(f"cfg {cfg} pair {i} layer {l}: {nm} differing labels, "
                  f"{nmoved} pixels with a different interval or tree upstream")


@pytest.mark.batch_inputs(3, 5)
@pytest.mark.parametrize("cfg", [3, 5])
def test_batched_teacher_forced_layers(H, orc, cfg):
    """Every layer of the full batched launch, with the spot pairs' upper-layer
    labels replaced by the oracle's before the interval prediction (the other
    pairs keep the GPU's): trees, tree intervals and pixel intervals bit-exact,
    the fused matching's aggregated costs within REL on sampled labels, labels
    equal except at oracle near-ties."""
    P = scenes.HDP_PARAMS[cfg]
    S, L, w = P["S"], P["L"], P["window"]
    pairs = scenes.workload_batch(cfg)
    shapes = [(p.shape[0], p.shape[1], p.dmax) for p in pairs]
    lv = H.level_shapes(shapes, S, L)
    off = [np.concatenate([[0], np.cumsum([h * wd for h, wd, _ in lv[l]])]) for l in range(L + 1)]
    lp, rp = H.pyramid_views(rgb_dev(*[p.left for p in pairs]), rgb_dev(*[p.right for p in pairs]),
                             shapes, S, L)
    spots = (0, len(pairs) // 2, len(pairs) - 1)
    opyr = {i: (orc.pyramid(pairs[i].left, S, L), orc.pyramid(pairs[i].right, S, L)) for i in spots}
    up_disp, oup = None, {}
    for l in range(L, -1, -1):
        if l == L:
            f = H.build_tree(lp[l], lv[l], l, level_order=False)
            glo = ghi = None
        else:
            forced = up_disp.clone()
            for i in spots:
                a, b = off[l + 1][i], off[l + 1][i + 1]
                forced[a:b] = torch.from_numpy(oup[i].ravel().astype(np.int32)).cuda()
            glo, ghi = H.predict_range(forced, lv[l + 1], lv[l], S, w)
            mw = min(S + 2 * w, max(d for _, _, d in lv[l]) + 1)
            f = H.build_tree(lp[l], lv[l], l, glo, ghi, max_width=mw, beta=P["beta"],
                             level_order=False)
        agg, disp = H.match_layer(lp[l], rp[l], lv[l], f)
        torch.cuda.synchronize()
        info = f.read_info()
        assert info[7] == 0 and info[6] == 0
        A = {k: f.array(k).cpu().numpy() for k in ("parent", "lo", "hi", "node", "row")}
        aggn, dispn = agg.cpu().numpy(), disp.cpu().numpy()
        for i in spots:
            Hl, Wl, dl = lv[l][i]
            a, n_l = off[l][i], Hl * Wl
            if l == L:
                plo = phi = None
            else:
                plo, phi = orc.predict_range(oup[i], Hl, Wl, S, w, dl)
                np.testing.assert_array_equal(glo.cpu().numpy()[a:a + n_l], plo.ravel())
                np.testing.assert_array_equal(ghi.cpu().numpy()[a:a + n_l], phi.ravel())
            labels = [0, dl // 2, dl] if l == L else [int(np.median(plo)), int(np.median(phi))]
            o = orc.stereo_level(opyr[i][0][l], opyr[i][1][l], dl, l, plo, phi, beta=P["beta"],
                                 sample_d=labels)
            par = A["parent"][a:a + n_l]
            np.testing.assert_array_equal(np.where(par >= 0, par - a, -1), o["parent"],
                                          err_msg=f"cfg {cfg} pair {i} layer {l} parent")
            np.testing.assert_array_equal(A["lo"][a:a + n_l], o["tree_lo"])
            np.testing.assert_array_equal(A["hi"][a:a + n_l], o["tree_hi"])
            rows = A["row"][a:a + n_l]
            got = np.full((len(labels), n_l), np.nan)
            tlo, thi = o["tree_lo"], o["tree_hi"]
            for k, x in enumerate(labels):
                ok = (x >= tlo) & (x <= thi)
                got[k, ok] = aggn[rows[ok], x - tlo[ok]]
            ref = o["sample_agg"]
            assert np.array_equal(np.isnan(got), np.isnan(ref))
            m = ~np.isnan(ref)
            err = np.abs(got[m] - ref[m]) / np.abs(ref[m])
            assert err.max() <= REL, f"cfg {cfg} pair {i} layer {l}: aggregate rel err {err.max():.3g}"
            d = dispn[a:a + n_l]
            od = o["disp"].ravel()
            mism = d != od
            near = (o["c2"] - o["c1"]) <= REL * np.abs(o["c1"])
            assert np.all(near[mism]), f"cfg {cfg} pair {i} layer {l}: label differences off near-ties"
            print(f"cfg {cfg} pair {i} layer {l}: {int(mism.sum())} near-tie label differences")
            oup[i] = o["disp"]
        up_disp = disp


def test_largest_pair_mst(H, orc):
    """One pair at the largest supported size (2^22 - 1 pixels limit): the MST
    and its level order bit-exact, one aggregated slice within tolerance."""
    Hh, Ww, d = 2047, 2048, 3
    pair = scenes.small_scene(99, Hh, Ww, d)
    shapes = [(Hh, Ww, d)]
    res = H.full_range(rgb_dev(pair.left), rgb_dev(pair.right), shapes, keep=True)
    o = orc.stereo_level(pair.left.astype(np.float64), pair.right.astype(np.float64), d, 0,
                         sample_d=[1])
    check_layer(H, orc, res, o, [1], "2047x2048")
