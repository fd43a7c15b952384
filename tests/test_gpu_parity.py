"""GPU parity: every stage of the HIP path against the FP64 oracle on the same
seeded inputs.  Trees, level order and ranges must match bit for bit; costs and
aggregated costs within 1e-5 relative of FP64; WTA labels identical except at
pixels whose two best oracle costs are within that tolerance (near-ties, counted).
"""

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


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rgb_dev(*imgs):
    return dev(np.concatenate([im.reshape(-1, 3) for im in imgs]))


def assert_rel(got, ref, rel=REL, what=""):
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    bad = np.abs(got - ref) > rel * np.abs(ref)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside {rel} rel; "
                             f"got {got.ravel()[i]} ref {ref.ravel()[i]}")


def forest_np(f):
    keys = ("parent", "depth", "tree", "lo", "hi", "row", "wgt", "order", "node", "prow",
            "heavy", "lc", "rw", "level_ptr")
    torch.cuda.synchronize()
    out = {k: f.array(k).cpu().numpy() for k in keys}
    out["info"] = f.read_info()
    return out


def volume_to_pixels(vol, F, D):
    """[n][width] rows of the forest layout -> [n][D] by pixel and label (NaN elsewhere)."""
    n, width = vol.shape
    out = np.full((n, D), np.nan)
    node = F["node"]
    for j in range(width):
        lab = F["lo"][node] + j
        ok = lab <= F["hi"][node]
        out[node[ok], lab[ok]] = vol[ok, j]
    return out


def check_forest(F, ref, n, what):
    info = F["info"]
    assert info[7] == 0, f"{what}: consistency guard tripped ({info[7]})"
    np.testing.assert_array_equal(F["parent"], ref["parent"], err_msg=f"{what} parent")
    np.testing.assert_array_equal(F["depth"], ref["depth"], err_msg=f"{what} depth")
    np.testing.assert_array_equal(F["tree"], ref["tree"], err_msg=f"{what} tree")
    np.testing.assert_array_equal(F["order"], ref["order"], err_msg=f"{what} order")
    nl = ref["n_levels"]
    assert info[0] == nl
    np.testing.assert_array_equal(F["level_ptr"][:nl + 1], ref["level_ptr"])
    assert_rel(F["wgt"], ref["wgt"], 1e-6, f"{what} wgt")
    # schedule invariants: rows are a permutation, chains contiguous, phases ordered
    node, row = F["node"], F["row"]
    assert np.array_equal(np.sort(node), np.arange(n))
    assert np.array_equal(row[node], np.arange(n))
    par_row = np.where(F["parent"][node] >= 0, row[np.maximum(F["parent"][node], 0)], -1)
    np.testing.assert_array_equal(F["prow"], par_row)
    hv = F["heavy"].astype(bool)
    assert np.all(F["prow"][hv] == np.flatnonzero(hv) - 1)


def run_level_oracle(orc, Lf, Rf, dmax, level, lo=None, hi=None, sigma=0.1, sample=None):
    """Oracle forest + full restricted volume + aggregated volume at one layer."""
    Hh, Ww = Lf.shape[:2]
    key = orc.edge_keys(Lf, level)
    in_tree, tlo, thi, _ = orc.kruskal(Hh, Ww, key, lo, hi)
    ref = orc.root_forest(Hh, Ww, in_tree, key, level)
    if lo is None:
        tlo = np.zeros(Hh * Ww, np.int32); thi = np.full(Hh * Ww, dmax, np.int32)
    cost = orc.cost_volume(Lf, Rf, dmax, tlo, thi)
    agg = orc.aggregate_twopass(ref["parent"], ref["wgt"], ref["order"], sigma,
                                np.nan_to_num(cost, nan=0.0))
    agg[np.isnan(cost)] = np.nan
    return dict(ref=ref, in_tree=in_tree, tlo=tlo, thi=thi, cost=cost, agg=agg, key=key)


def check_wta(disp, agg_ref, tlo, thi, what):
    import oracle.oracle as O
    d_ref, c1, c2 = O.wta(np.nan_to_num(agg_ref, nan=np.inf), tlo, thi)
    mism = disp != d_ref
    near = (c2 - c1) <= REL * np.abs(c1)
    assert np.all(near[mism]), f"{what}: {int((mism & ~near).sum())} WTA mismatches off near-ties"
    return int(mism.sum()), int(near.sum())


# --- pyramid -----------------------------------------------------------------------

@pytest.mark.parametrize("Hh,Ww", [(120, 160), (37, 53), (1, 9), (9, 1), (1, 1)])
def test_pyramid_exact(H, orc, Hh, Ww):
    img = np.random.default_rng(Hh * 1000 + Ww).integers(0, 256, (Hh, Ww, 3)).astype(np.uint8)
    L = 3
    lv = H.pyramid(rgb_dev(img), [(Hh, Ww, 15)], 2, L)
    ref = orc.pyramid(img, 2, L)
    for l in range(L + 1):
        got = lv[l].cpu().numpy()[:, :3].reshape(ref[l].shape)
        np.testing.assert_array_equal(got, ref[l].astype(np.float32))


def test_pyramid_unaligned_input_and_batch_rows(H, orc):
    """Layer 0 read four pixels per thread from 32-bit words, and pixel by
    pixel where the buffer is not 4-byte aligned or the words would leave it:
    both give the oracle's layer (gx included) on a batch whose pairs start at
    every offset modulo 4 and rows of odd widths."""
    shapes = [(5, 7, 15), (3, 13, 15), (6, 1, 15), (4, 9, 15), (2, 3, 15)]
    rng = np.random.default_rng(77)
    imgs = [rng.integers(0, 256, (h, w, 3)).astype(np.uint8) for h, w, _ in shapes]
    flat = np.concatenate([im.reshape(-1, 3) for im in imgs])
    base = torch.zeros(flat.size + 8, dtype=torch.uint8, device="cuda")
    for shift in (0, 1, 2, 3):
        view = base[shift:shift + flat.size]
        view.copy_(torch.from_numpy(flat.ravel()).cuda())
        lv = H.pyramid(view.view(-1, 3), shapes, 2, 0)
        got = lv[0].cpu().numpy()
        off = 0
        for im in imgs:
            h, w = im.shape[:2]
            g = got[off:off + h * w].reshape(h, w, 4)
            off += h * w
            np.testing.assert_array_equal(g[..., :3], im.astype(np.float32), err_msg=f"shift {shift}")
            S = im.astype(np.int64).sum(axis=2)
            right = np.concatenate([S[:, 1:], S[:, -1:]], axis=1)
            left = np.concatenate([S[:, :1], S[:, :-1]], axis=1)
            np.testing.assert_array_equal(g[..., 3], (right - left).astype(np.float32),
                                          err_msg=f"shift {shift}")


def test_pyramid_views_and_gradient(H, orc):
    """Both views in one call equal two single-view calls; the gx channel of
    every layer is S(x+1) - S(x-1) of the channel sums S (replicated border),
    exact because layer values are dyadic means."""
    rng = np.random.default_rng(77)
    shapes = [(45, 70, 31), (17, 5, 15)]
    imgs = [rng.integers(0, 256, (h, w, 3)).astype(np.uint8) for h, w, _ in shapes]
    imgs_r = [rng.integers(0, 256, (h, w, 3)).astype(np.uint8) for h, w, _ in shapes]
    L = 3
    lv_l, lv_r = H.pyramid_views(rgb_dev(*imgs), rgb_dev(*imgs_r), shapes, 2, L)
    single_l = H.pyramid(rgb_dev(*imgs), shapes, 2, L)
    single_r = H.pyramid(rgb_dev(*imgs_r), shapes, 2, L)
    for l in range(L + 1):
        np.testing.assert_array_equal(lv_l[l].cpu().numpy(), single_l[l].cpu().numpy())
        np.testing.assert_array_equal(lv_r[l].cpu().numpy(), single_r[l].cpu().numpy())
    off = 0
    got = [lv_l[l].cpu().numpy() for l in range(L + 1)]
    offs = [0] * (L + 1)
    for img in imgs:
        ref = orc.pyramid(img, 2, L)
        for l in range(L + 1):
            h, w = ref[l].shape[:2]
            g = got[l][offs[l]:offs[l] + h * w].reshape(h, w, 4)
            offs[l] += h * w
            np.testing.assert_array_equal(g[..., :3], ref[l].astype(np.float32))
            S = ref[l].sum(axis=2)
            right = np.concatenate([S[:, 1:], S[:, -1:]], axis=1)
            left = np.concatenate([S[:, :1], S[:, :-1]], axis=1)
            np.testing.assert_array_equal(g[..., 3], (right - left).astype(np.float32))


# --- trees -------------------------------------------------------------------------

@pytest.mark.parametrize("Hh,Ww,seed", [(120, 160, 1), (31, 47, 2), (1, 64, 3), (64, 1, 4),
                                        (1, 1, 5), (2, 2, 6), (200, 300, 7)])
def test_mst_bit_exact(H, orc, Hh, Ww, seed):
    pair = scenes.small_scene(seed, Hh, Ww, 15)
    lv = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, 15)], 2, 0)
    f = H.build_tree(lv[0], [(Hh, Ww, 15)], 0)
    F = forest_np(f)
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, _, _, _ = orc.kruskal(Hh, Ww, key)
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    check_forest(F, ref, Hh * Ww, f"MST {Hh}x{Ww}")
    assert F["info"][2] == 1  # one tree


def test_mst_top_layer_tail_global_mode(H, orc):
    # A layer without intervals and with few tile-border pixels launches no
    # full-grid rounds.  Here every pixel takes the colour of its distance to
    # the nearest 32-pixel tile border, so pixels facing each other across a
    # border match and most border pixels wait on their crossing edge in the
    # tile-local phase: more live edges remain than the LDS tail holds, and the
    # tail finishes the forest in its global-memory mode.
    Hh, Ww = 160, 192
    yy, xx = np.mgrid[0:Hh, 0:Ww]
    dx = np.minimum(xx % 32, 31 - xx % 32)
    dy = np.minimum(yy % 32, 31 - yy % 32)
    base = np.random.default_rng(5).integers(0, 256, (16, 16, 3), dtype=np.uint8)
    img = np.ascontiguousarray(base[dy, dx])
    lv = H.pyramid(rgb_dev(img), [(Hh, Ww, 15)], 2, 0)
    f = H.build_tree(lv[0], [(Hh, Ww, 15)], 0)
    F = forest_np(f)
    key = orc.edge_keys(img.astype(np.float64), 0)
    in_tree, _, _, _ = orc.kruskal(Hh, Ww, key)
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    check_forest(F, ref, Hh * Ww, "MST tile-mirrored 160x192")
    assert F["info"][H.INFO["live_edges"]] > 6144, F["info"][H.INFO["live_edges"]]


@pytest.mark.parametrize("level", [1, 2, 3])
def test_mst_upper_levels_bit_exact(H, orc, level):
    pair = scenes.small_scene(11, 97, 131, 31)
    lv = H.pyramid(rgb_dev(pair.left), [(97, 131, 31)], 2, 3)
    shp = H.level_shapes([(97, 131, 31)], 2, 3)[level]
    f = H.build_tree(lv[level], shp, level)
    F = forest_np(f)
    ref_img = orc.pyramid(pair.left, 2, 3)[level]
    key = orc.edge_keys(ref_img, level)
    in_tree, _, _, _ = orc.kruskal(shp[0][0], shp[0][1], key)
    ref = orc.root_forest(shp[0][0], shp[0][1], in_tree, key, level)
    check_forest(F, ref, shp[0][0] * shp[0][1], f"MST level {level}")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hdpf_bit_exact(H, orc, seed):
    Hh, Ww, dmax, S, w = 96, 128, 63, 2, 4
    pair = scenes.small_scene(20 + seed, Hh, Ww, dmax)
    up = np.random.default_rng(seed).integers(0, dmax // 2 + 1, ((Hh + 1) // 2, (Ww + 1) // 2))
    # blocky parent labels so that equal-interval regions are large
    up = np.kron(up[::4, ::4], np.ones((4, 4), int))[:up.shape[0], :up.shape[1]]
    lo, hi = orc.predict_range(up, Hh, Ww, S, w, dmax)
    lv = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, dmax)], 2, 0)
    f = H.build_tree(lv[0], [(Hh, Ww, dmax)], 0, dev(lo.ravel(), torch.int32),
                     dev(hi.ravel(), torch.int32), max_width=S + 2 * w, beta=(19, 20))
    F = forest_np(f)
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, tlo, thi, _ = orc.kruskal(Hh, Ww, key, lo, hi, beta=(19, 20))
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    check_forest(F, ref, Hh * Ww, "HDPF")
    np.testing.assert_array_equal(F["lo"], tlo)
    np.testing.assert_array_equal(F["hi"], thi)
    assert F["info"][6] == 0


@pytest.mark.parametrize("case", ["beta35_w4", "beta35_w8", "beta12_batch2"])
def test_hdpf_literal_outside_regime(H, orc, case):
    """Outside the exact regime (beta = 3/5, the small-image setting of
    Section 4.1; wide windows) the forest is the one of the sequential Kruskal
    process with both DT rules on the current tree intervals: parents, trees,
    depths, level order, weights and each pixel's tree interval bit-exact
    against the oracle's literal process."""
    S, dmax = 2, 63
    if case == "beta12_batch2":
        shapes, w, beta = [(40, 56, dmax), (23, 31, dmax)], 4, (1, 2)
    else:
        shapes, w, beta = [(48, 64, dmax)], (4 if case == "beta35_w4" else 8), (3, 5)
    pairs = [scenes.small_scene(610 + i, h, wd, d) for i, (h, wd, d) in enumerate(shapes)]
    los, his, refs = [], [], []
    for i, (pair, (h, wd, _)) in enumerate(zip(pairs, shapes)):
        up = np.random.default_rng(30 + i).integers(0, dmax // 2 + 1, ((h + 1) // 2, (wd + 1) // 2))
        up = np.kron(up[::3, ::3], np.ones((3, 3), int))[:up.shape[0], :up.shape[1]]
        lo, hi = orc.predict_range(up, h, wd, S, w, dmax)
        key = orc.edge_keys(pairs[i].left.astype(np.float64), 0)
        in_tree, tlo, thi, _ = orc.kruskal(h, wd, key, lo, hi, beta=beta)
        refs.append((orc.root_forest(h, wd, in_tree, key, 0), tlo, thi))
        los.append(lo.ravel()); his.append(hi.ravel())
    lv = H.pyramid(rgb_dev(*[p.left for p in pairs]), shapes, 2, 0)
    lo_d = dev(np.concatenate(los), torch.int32); hi_d = dev(np.concatenate(his), torch.int32)
    mw = S + 2 * w
    assert beta[0] * mw <= beta[1] * (mw - 1)  # outside the regime
    f = H.build_tree(lv[0], shapes, 0, lo_d, hi_d, max_width=mw, beta=beta)
    assert f.width == dmax + 1
    F = forest_np(f)
    assert F["info"][6] == 0
    off = 0
    for i, ((h, wd, _), (ref, tlo, thi)) in enumerate(zip(shapes, refs)):
        n = h * wd
        sl = slice(off, off + n)
        # pixel ids of pair i are offset by the pixels of the pairs before it
        np.testing.assert_array_equal(F["parent"][sl], np.where(ref["parent"] >= 0,
                                                                ref["parent"] + off, -1))
        np.testing.assert_array_equal(F["tree"][sl], ref["tree"] + off)
        np.testing.assert_array_equal(F["depth"][sl], ref["depth"])
        assert_rel(F["wgt"][sl], ref["wgt"], 1e-6, f"{case} pair {i} wgt")
        np.testing.assert_array_equal(F["lo"][sl], tlo)
        np.testing.assert_array_equal(F["hi"][sl], thi)
        if len(shapes) == 1:
            check_forest(F, ref, n, f"literal HDPF {case}")
        off += n
    # some trees merged across different intervals (the case the regime excludes)
    assert np.any(F["hi"] - F["lo"] + 1 > mw) or np.any(
        (F["lo"] != np.concatenate(los)) | (F["hi"] != np.concatenate(his)))


@pytest.mark.parametrize("Hh,Ww", [(1, 1), (1, 17), (17, 1), (2, 2), (3, 40)])
def test_hdpf_literal_degenerate_shapes(H, orc, Hh, Ww):
    """The literal disparity forest on degenerate grids (a single pixel, one
    row, one column, 2x2, a thin strip) with random intervals and beta = 1/2:
    bit-exact against the oracle's literal process."""
    dmax = 15
    rng = np.random.default_rng(Hh * 100 + Ww)
    img = rng.integers(0, 256, (Hh, Ww, 3)).astype(np.uint8)
    lo = rng.integers(0, 10, Hh * Ww).astype(np.int32)
    hi = np.minimum(lo + rng.integers(0, 6, Hh * Ww), dmax).astype(np.int32)
    shapes = [(Hh, Ww, dmax)]
    lv = H.pyramid(rgb_dev(img), shapes, 2, 0)
    f = H.build_tree(lv[0], shapes, 0, dev(lo, torch.int32), dev(hi, torch.int32),
                     max_width=6, beta=(1, 2))
    F = forest_np(f)
    key = orc.edge_keys(img.astype(np.float64), 0)
    in_tree, tlo, thi, _ = orc.kruskal(Hh, Ww, key, lo.reshape(Hh, Ww), hi.reshape(Hh, Ww),
                                       beta=(1, 2))
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    check_forest(F, ref, Hh * Ww, f"literal {Hh}x{Ww}")
    np.testing.assert_array_equal(F["lo"], tlo)
    np.testing.assert_array_equal(F["hi"], thi)
    assert F["info"][6] == 0


def test_hdp_literal_end_to_end_small(H, orc):
    """The whole loop with beta = 3/5 (outside the regime at every layer below
    the top) on the GPU against the oracle's literal loop: labels identical
    except at near-ties or where an interval upstream differs."""
    pair = scenes.small_scene(640, 48, 64, 31)
    res = H.hdp_stereo(rgb_dev(pair.left), rgb_dev(pair.right), [(48, 64, 31)], S=2, L=2,
                       window=2, beta=(3, 5))
    ores = orc.hdp_stereo(pair.left, pair.right, 31, S=2, L=2, window=2, beta=(3, 5))
    for l in (2, 1, 0):
        g = res[l].disp.cpu().numpy(); o = ores[l]["disp"].ravel()
        gap = (ores[l]["c2"] - ores[l]["c1"]) / ores[l]["c1"]
        mism = g != o
        if l < 2:
            same_int = ((res[l].pix_lo.cpu().numpy() == ores[l]["pix_lo"].ravel()) &
                        (res[l].pix_hi.cpu().numpy() == ores[l]["pix_hi"].ravel()))
        else:
            same_int = np.ones_like(mism)
        assert np.all(gap[mism & same_int] <= REL), f"layer {l}: unexplained mismatches"



def test_hdp_border_clamp_end_to_end_small(H, orc):
    """The whole loop with the clamped border (labels past the left edge
    compared with the row's first pixel) on the GPU against the oracle's loop
    with the same policy: labels identical except at near-ties or where an
    interval upstream differs."""
    pair = scenes.small_scene(641, 48, 80, 31)
    prm = (0.89, 7.0, 0.11, 2.0, 1)
    res = H.hdp_stereo(rgb_dev(pair.left), rgb_dev(pair.right), [(48, 80, 31)], S=2, L=2,
                       window=2, params=H.cost_params(*prm))
    ores = orc.hdp_stereo(pair.left, pair.right, 31, S=2, L=2, window=2, prm=prm)
    for l in (2, 1, 0):
        g = res[l].disp.cpu().numpy(); o = ores[l]["disp"].ravel()
        gap = (ores[l]["c2"] - ores[l]["c1"]) / ores[l]["c1"]
        mism = g != o
        if l < 2:
            same_int = ((res[l].pix_lo.cpu().numpy() == ores[l]["pix_lo"].ravel()) &
                        (res[l].pix_hi.cpu().numpy() == ores[l]["pix_hi"].ravel()))
        else:
            same_int = np.ones_like(mism)
        assert np.all(gap[mism & same_int] <= REL), f"layer {l}: unexplained mismatches"
    # the policy changes the result: the saturated border gives other labels somewhere
    sat = H.hdp_stereo(rgb_dev(pair.left), rgb_dev(pair.right), [(48, 80, 31)], S=2, L=2,
                       window=2)
    assert not np.array_equal(sat[0].disp.cpu().numpy(), res[0].disp.cpu().numpy())


# --- cost, aggregation, WTA ------------------------------------------------------------

@pytest.mark.parametrize("Hh,Ww,dmax,seed", [(120, 160, 15, 1001), (45, 70, 31, 7),
                                             (33, 257, 255, 8), (17, 5, 0, 9)])
def test_full_range_layer(H, orc, Hh, Ww, dmax, seed):
    pair = scenes.small_scene(seed, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    agg = H.aggregate(f, cost, 0.1)
    disp = H.wta(agg, shapes, f)
    F = forest_np(f)
    o = run_level_oracle(orc, pair.left.astype(np.float64), pair.right.astype(np.float64),
                         dmax, 0)
    check_forest(F, o["ref"], Hh * Ww, "full-range tree")
    D = dmax + 1
    assert_rel(volume_to_pixels(cost.cpu().numpy(), F, D), o["cost"], REL, "cost")
    assert_rel(volume_to_pixels(agg.cpu().numpy(), F, D), o["agg"], REL, "aggregate")
    nm, nt = check_wta(disp.cpu().numpy(), o["agg"], o["tlo"], o["thi"], "WTA")
    print(f"WTA mismatches {nm} (near-ties {nt})")


def test_dense_cost_and_wta(H, orc):
    Hh, Ww, dmax = 40, 60, 23
    pair = scenes.small_scene(31, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    cost = H.cost_volume(lp[0], rp[0], shapes).cpu().numpy()
    ref = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax)
    assert_rel(cost, ref, REL, "dense cost")
    disp = H.wta(dev(cost), shapes).cpu().numpy()
    d_ref, c1, c2 = orc.wta(cost.astype(np.float64))
    np.testing.assert_array_equal(disp, d_ref)


@pytest.mark.parametrize("level,seed", [(0, 1), (1, 2), (2, 3)])
def test_hdp_layer_stagewise(H, orc, level, seed):
    """Layer l of HDP with the ORACLE's layer-(l+1) disparities as input."""
    Hh, Ww, dmax, S, w, L = 96, 128, 63, 2, 4, 3
    pair = scenes.small_scene(40 + seed, Hh, Ww, dmax)
    ores = orc.hdp_stereo(pair.left, pair.right, dmax, S=S, L=L, window=w, want_forest=True)
    lvs = H.level_shapes([(Hh, Ww, dmax)], S, L)
    lp = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, dmax)], S, L)
    rp = H.pyramid(rgb_dev(pair.right), [(Hh, Ww, dmax)], S, L)
    up = dev(ores[level + 1]["disp"].ravel(), torch.int32)
    lo, hi = H.predict_range(up, lvs[level + 1], lvs[level], S, w)
    np.testing.assert_array_equal(lo.cpu().numpy(), ores[level]["pix_lo"].ravel())
    np.testing.assert_array_equal(hi.cpu().numpy(), ores[level]["pix_hi"].ravel())
    dl = lvs[level][0][2]
    r = H.stereo_level(lp[level], rp[level], lvs[level], level, lo, hi,
                       max_width=min(S + 2 * w, dl + 1), keep=True)
    F = forest_np(r.forest)
    assert F["info"][7] == 0
    np.testing.assert_array_equal(F["parent"], ores[level]["parent"])
    np.testing.assert_array_equal(F["order"], ores[level]["order"])
    np.testing.assert_array_equal(F["lo"], ores[level]["tree_lo"])
    np.testing.assert_array_equal(F["hi"], ores[level]["tree_hi"])
    Lf = orc.pyramid(pair.left, S, L)[level]; Rf = orc.pyramid(pair.right, S, L)[level]
    o = run_level_oracle(orc, Lf, Rf, dl, level, ores[level]["pix_lo"], ores[level]["pix_hi"])
    assert_rel(volume_to_pixels(r.agg.cpu().numpy(), F, dl + 1), o["agg"], REL, "HDP aggregate")
    nm, nt = check_wta(r.disp.cpu().numpy(), o["agg"], o["tlo"], o["thi"], "HDP WTA")
    print(f"level {level}: WTA mismatches {nm} (near-ties {nt})")


def test_hdp_end_to_end_small(H, orc):
    """Whole loop on the GPU vs the whole loop in the oracle (config-1 sized)."""
    pair = scenes.workload(1)
    Hh, Ww = pair.shape
    res = H.hdp_stereo(rgb_dev(pair.left), rgb_dev(pair.right), [(Hh, Ww, 15)], S=2, L=2,
                       window=2)
    ores = orc.hdp_stereo(pair.left, pair.right, 15, S=2, L=2, window=2)
    for l in (2, 1, 0):
        g = res[l].disp.cpu().numpy(); o = ores[l]["disp"].ravel()
        gap = (ores[l]["c2"] - ores[l]["c1"]) / ores[l]["c1"]
        mism = g != o
        # a mismatch must come from a near-tie here or from a different interval upstream
        if l < 2:
            same_int = ((res[l].pix_lo.cpu().numpy() == ores[l]["pix_lo"].ravel()) &
                        (res[l].pix_hi.cpu().numpy() == ores[l]["pix_hi"].ravel()))
        else:
            same_int = np.ones_like(mism)
        assert np.all(gap[mism & same_int] <= REL), f"layer {l}: unexplained mismatches"
        print(f"layer {l}: {int(mism.sum())} label mismatches, {int((gap <= REL).sum())} near-ties")


def _three_steps(H, lp, rp, shapes, f, sigma=0.1):
    cost = H.cost_volume(lp, rp, shapes, f)
    agg = H.aggregate(f, cost, sigma)
    return agg, H.wta(agg, shapes, f)


@pytest.mark.parametrize("case", ["hdp_layer0", "hdp_layer1_batch", "top_width32", "wide_width64"])
def test_fused_match_layer_equals_three_steps(H, case):
    """hdp_match_layer (fused cost in the up pass for rows of at most 64 labels
    or up to 256 in fours, the right image packed from 64 labels on; the
    winner-takes-all fused into the down pass) gives bit for bit the aggregated
    volume and the labels of hdp_cost_volume + hdp_aggregate + hdp_wta on the
    same forest."""
    S, L, w = 2, 3, 4
    if case == "hdp_layer1_batch":
        shapes = [(96, 128, 63), (37, 53, 31), (1, 40, 15)]
    elif case == "wide_width64":
        shapes = [(45, 70, 63)]
    elif case == "top_width32":
        shapes = [(70, 90, 31)]
    else:
        shapes = [(96, 128, 63)]
    pairs = [scenes.small_scene(500 + i, h, wd, d) for i, (h, wd, d) in enumerate(shapes)]
    Lr, Rr = rgb_dev(*[p.left for p in pairs]), rgb_dev(*[p.right for p in pairs])
    if case in ("top_width32", "wide_width64"):
        lp, rp = H.pyramid_views(Lr, Rr, shapes, S, 0)
        lv, level, lo, hi, mw = shapes, 0, None, None, 0
        lp, rp = lp[0], rp[0]
    else:
        level = 1 if case == "hdp_layer1_batch" else 0
        lvs = H.level_shapes(shapes, S, L)
        res = H.hdp_stereo(Lr, Rr, shapes, S=S, L=L, window=w)
        lo, hi = H.predict_range(res[level + 1].disp, lvs[level + 1], lvs[level], S, w)
        lps, rps = H.pyramid_views(Lr, Rr, shapes, S, L)
        lp, rp, lv = lps[level], rps[level], lvs[level]
        mw = min(S + 2 * w, max(d for _, _, d in lv) + 1)
    f = H.build_tree(lp, lv, level, lo, hi, max_width=mw)
    agg3, disp3 = _three_steps(H, lp, rp, lv, f)
    aggf, dispf = H.match_layer(lp, rp, lv, f)
    torch.cuda.synchronize()
    assert f.read_info()[7] == 0
    assert torch.equal(aggf, agg3), f"{case}: aggregated volumes differ"
    assert torch.equal(dispf, disp3), f"{case}: labels differ"


@pytest.mark.parametrize("case", ["w256_layer0", "w64_layer2", "w256_fallback", "w128_batch2"])
def test_packed_right_image_equals_three_steps(H, case):
    """Rows of >= 64 labels: the fused up pass reads the right image packed in
    8 bytes a pixel (exact for pyramid pixels: multiples of 4^-l).  Its results
    equal those of the three separate steps bit for bit: at layer 0 (256
    labels), at layer 2 (64 labels, pixels in sixteenths), on a batch of two
    pairs, and with pixels that do not pack (fractional or out-of-range values:
    read as FP32 instead)."""
    if case == "w64_layer2":
        shapes, level = [(120, 200, 255)], 2
    elif case == "w128_batch2":
        shapes, level = [(30, 150, 127), (25, 90, 127)], 0
    else:
        shapes, level = [(40, 300, 255)], 0
    pairs = [scenes.small_scene(520 + i, h, wd, d) for i, (h, wd, d) in enumerate(shapes)]
    Lr, Rr = rgb_dev(*[p.left for p in pairs]), rgb_dev(*[p.right for p in pairs])
    lps, rps = H.pyramid_views(Lr, Rr, shapes, 2, level)
    lv = H.level_shapes(shapes, 2, level)[level]
    lp, rp = lps[level], rps[level]
    if case == "w256_fallback":
        rp = rp.clone()
        px = rp.view(-1, 4)
        px[::5, 0] += 0.25       # not a whole number: no exact packing
        px[7, 1] = 20000.0       # beyond the packed field
    f = H.build_tree(lp, lv, level)
    assert f.width >= 64
    agg3, disp3 = _three_steps(H, lp, rp, lv, f)
    aggf, dispf = H.match_layer(lp, rp, lv, f)
    torch.cuda.synchronize()
    assert f.read_info()[7] == 0
    assert torch.equal(aggf, agg3), f"{case}: aggregated volumes differ"
    assert torch.equal(dispf, disp3), f"{case}: labels differ"


@pytest.mark.parametrize("width_case", ["hdp_w10", "full_w64"])
def test_border_policy_clamp(H, orc, width_case):
    """Border policy 1 (a label past the left border compared with the row's
    first pixel): the cost volume within 1e-5 of the oracle's with the same
    policy, and the fused matching bit for bit equal to the three separate
    steps (FP32 right pixels on HDP windows, packed ones on 64-label rows)."""
    Hh, Ww, dmax = 40, 56, 63
    pair = scenes.small_scene(91, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    Lr, Rr = rgb_dev(pair.left), rgb_dev(pair.right)
    lp, rp = H.pyramid_views(Lr, Rr, shapes, 2, 0)
    if width_case == "hdp_w10":
        lo = np.clip(np.arange(Hh * Ww) % 37 - 4, 0, dmax).astype(np.int32)
        hi = np.minimum(lo + 9, dmax).astype(np.int32)
        f = H.build_tree(lp[0], shapes, 0, dev(lo, torch.int32), dev(hi, torch.int32),
                         max_width=10)
    else:
        lo = np.zeros(Hh * Ww, np.int32); hi = np.full(Hh * Ww, dmax, np.int32)
        f = H.build_tree(lp[0], shapes, 0)
    p = H.cost_params(border=1)
    cost = H.cost_volume(lp[0], rp[0], shapes, f, params=p)
    F = forest_np(f)
    got = volume_to_pixels(cost.cpu().numpy(), F, dmax + 1)
    tlo, thi = F["lo"], F["hi"]
    ref = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax,
                          tlo.reshape(Hh, Ww), thi.reshape(Hh, Ww), prm=orc.COST_PARAMS + (1,))
    m = ~np.isnan(ref)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert_rel(got[m], ref[m], REL, f"border 1 cost {width_case}")
    # the policies differ exactly where the label passes the left border
    ref0 = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax,
                           tlo.reshape(Hh, Ww), thi.reshape(Hh, Ww))
    x = np.arange(Hh * Ww) % Ww
    past = np.arange(dmax + 1)[None, :] > x[:, None]
    assert np.array_equal(ref0[m & ~past], ref[m & ~past])
    agg = H.aggregate(f, cost, 0.1)
    disp = H.wta(agg, shapes, f)
    aggf, dispf = H.match_layer(lp[0], rp[0], shapes, f, params=p)
    torch.cuda.synchronize()
    assert torch.equal(aggf, agg) and torch.equal(dispf, disp)


def test_workspace_reuse_no_stale_rows(H):
    """Only the rows a tile polls are marked unwritten before a pass; a call on
    a workspace that holds another input's rows must still give the results of
    a fresh workspace, bit for bit (HDP layer 0 and the full-range top layer)."""
    shapes = [(96, 128, 63)]
    S, L, w = 2, 3, 4
    lvs = H.level_shapes(shapes, S, L)
    runs = []
    for seed in (11, 12):
        p = scenes.small_scene(seed, *shapes[0])
        Lr, Rr = rgb_dev(p.left), rgb_dev(p.right)
        res = H.hdp_stereo(Lr, Rr, shapes, S=S, L=L, window=w)
        lps, rps = H.pyramid_views(Lr, Rr, shapes, S, L)
        runs.append((res, lps, rps))
    shared = H.Workspace()
    for level in (0, L):
        for k in (0, 1):  # input 0 then input 1 on the shared workspace
            res, lps, rps = runs[k]
            aggs, disps = H.match_layer(lps[level], rps[level], lvs[level], res[level].forest,
                                        ws=shared)
        res, lps, rps = runs[1]
        aggf, dispf = H.match_layer(lps[level], rps[level], lvs[level], res[level].forest,
                                    ws=H.Workspace())
        torch.cuda.synchronize()
        assert torch.equal(aggs, aggf), f"layer {level}: stale rows in the aggregated volume"
        assert torch.equal(disps, dispf), f"layer {level}: stale rows in the labels"


@pytest.mark.parametrize("Hh,Ww,dmax", [(70, 90, 31), (45, 70, 127)])
def test_aggregate_reproducible(H, Hh, Ww, dmax):
    """Two aggregations of the same cost give the same bits (narrow rows with
    32 labels, wide rows with 128): a tile's carry does not depend on which of
    its predecessors had finished."""
    pair = scenes.small_scene(77, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp, rp = H.pyramid_views(rgb_dev(pair.left), rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    runs = [H.aggregate(f, cost, 0.1).clone() for _ in range(4)]
    torch.cuda.synchronize()
    for r in runs[1:]:
        assert torch.equal(r, runs[0])


def test_batched_matches_single(H):
    """Two uneven pairs in one call give the per-pair results of single calls."""
    shapes = [(50, 70, 31), (33, 41, 15)]
    pairs = [scenes.small_scene(60 + i, h, w, d) for i, (h, w, d) in enumerate(shapes)]
    rb = H.hdp_stereo(rgb_dev(*[p.left for p in pairs]), rgb_dev(*[p.right for p in pairs]),
                      shapes, S=2, L=2, window=2)
    off = 0
    for p, (h, w, d) in zip(pairs, shapes):
        rs = H.hdp_stereo(rgb_dev(p.left), rgb_dev(p.right), [(h, w, d)], S=2, L=2, window=2)
        np.testing.assert_array_equal(rb[0].disp.cpu().numpy()[off:off + h * w],
                                      rs[0].disp.cpu().numpy())
        off += h * w


# --- adjoint --------------------------------------------------------------------------

def test_adjoint_matches_oracle(H, orc):
    """dL/dC, dL/dw and dL/dsigma of L = sum g * agg against the oracle's two-pass
    adjoint (itself pinned to the dense gradient and FP64 finite differences).
    The gradients are sums of mixed-sign terms, so the bound is 1e-5 of the same
    sums taken over absolute values (what FP32 rounding of the terms scales with)."""
    Hh, Ww, dmax, sigma = 32, 48, 7, 0.1
    pair = scenes.small_scene(77, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    agg, up = H.aggregate(f, cost, sigma, keep_up=True)
    g = torch.from_numpy(np.random.default_rng(3).normal(size=cost.shape).astype(np.float32)).cuda()
    gc, gw, gs = H.aggregate_backward(f, cost, agg, g, sigma, up=up)
    gc2, gw2, gs2 = H.aggregate_backward(f, cost, agg, g, sigma, up=None)
    F = forest_np(f)
    node = F["node"]
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, _, _, _ = orc.kruskal(Hh, Ww, key)
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    par, wg, od = ref["parent"], ref["wgt"], ref["order"]
    C = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax)
    Gp = np.zeros_like(C); Gp[node] = g.cpu().numpy().astype(np.float64)
    dC, dw, ds = orc.aggregate_backward_twopass(par, wg, od, sigma, C, Gp)
    # magnitudes: the same sums over |g|
    Aabs, Uabs = orc.aggregate_twopass(par, wg, od, sigma, np.abs(Gp), want_up=True)
    AC, UC = orc.aggregate_twopass(par, wg, od, sigma, C, want_up=True)
    got = np.zeros_like(C); got[node] = gc.cpu().numpy()
    assert np.all(np.abs(got - dC) <= REL * Aabs), np.max(np.abs(got - dC) / Aabs)
    s = np.where(par >= 0, np.exp(-wg / sigma), 0.0)
    pp = np.maximum(par, 0)
    B = np.sum(Uabs * (AC[pp] + s[:, None] * UC) + UC * (Aabs[pp] + s[:, None] * Uabs), axis=1)
    B = np.where(par >= 0, B * s / sigma, 0.0)
    gwn = gw.cpu().numpy()
    assert np.all(np.abs(gwn - dw) <= REL * B + 1e-30), np.max(np.abs(gwn - dw) / np.maximum(B, 1e-30))
    Bs = float(np.sum(B * wg / sigma))
    assert abs(float(gs.cpu()) - ds) <= REL * Bs, (float(gs.cpu()), ds, Bs)
    # recomputing U instead of reusing the forward's gives the same gradients
    np.testing.assert_array_equal(gc2.cpu().numpy(), gc.cpu().numpy())


def adjoint_reference(orc, par, wg, od, sigma, C, G):
    """Oracle adjoint (two-pass, pinned to the dense gradient and FP64 finite
    differences) and the rounding scale of each gradient: the same sums taken
    over absolute values."""
    dC, dw, ds = orc.aggregate_backward_twopass(par, wg, od, sigma, C, G)
    Aabs, Uabs = orc.aggregate_twopass(par, wg, od, sigma, np.abs(G), want_up=True)
    AC, UC = orc.aggregate_twopass(par, wg, od, sigma, C, want_up=True)
    s = np.where(par >= 0, np.exp(-wg / sigma), 0.0)
    pp = np.maximum(par, 0)
    B = np.sum(Uabs * (AC[pp] + s[:, None] * UC) + UC * (Aabs[pp] + s[:, None] * Uabs), axis=1)
    B = np.where(par >= 0, B * s / sigma, 0.0)
    return dict(dC=dC, dw=dw, ds=ds, bC=Aabs, bw=B, bs=float(np.sum(B * wg / sigma)))


def check_adjoint(got_c, got_w, got_s, ref, what, mask=None):
    """Within REL of the magnitude sums (the FP32 rounding bound of a sum of
    mixed-sign terms); also prints how the relative error behaves where the
    reference is not small (|ref| >= 1e-3 of its largest value)."""
    m = np.ones(ref["dC"].shape, bool) if mask is None else mask
    ec = np.abs(got_c - ref["dC"])[m]
    assert np.all(ec <= REL * ref["bC"][m]), f"{what} dC: {np.max(ec / ref['bC'][m]):.3g}"
    ew = np.abs(got_w - ref["dw"])
    assert np.all(ew <= REL * ref["bw"] + 1e-30), f"{what} dw: {np.max(ew / np.maximum(ref['bw'], 1e-30)):.3g}"
    assert abs(got_s - ref["ds"]) <= REL * ref["bs"], (what, got_s, ref["ds"], ref["bs"])
    for name, g_, r_ in (("dC", got_c[m], ref["dC"][m]), ("dw", got_w, ref["dw"])):
        big = np.abs(r_) >= 1e-3 * np.max(np.abs(r_))
        rel = np.abs(g_ - r_)[big] / np.abs(r_)[big]
        print(f"{what} {name}: rel err where |ref| >= 1e-3 max: max {rel.max():.3g}, "
              f"99.9% {np.quantile(rel, 0.999):.3g}, above 1e-5: {int((rel > 1e-5).sum())} of {rel.size}")
    if ref["ds"] != 0.0:
        print(f"{what} dsigma rel err {abs(got_s - ref['ds']) / abs(ref['ds']):.3g}")


def test_adjoint_hdp_forest(H, orc):
    """The adjoint on a disparity forest with many trees and narrow per-tree
    label windows (the shape of the batched backward over HDP layers): dC inside
    every tree interval, dw per node and dsigma against the oracle."""
    Hh, Ww, dmax, S, w, sigma = 48, 64, 31, 2, 2, 0.1
    pair = scenes.small_scene(88, Hh, Ww, dmax)
    up = np.random.default_rng(8).integers(0, dmax // 2 + 1, ((Hh + 1) // 2, (Ww + 1) // 2))
    up = np.kron(up[::3, ::3], np.ones((3, 3), int))[:up.shape[0], :up.shape[1]]
    lo, hi = orc.predict_range(up, Hh, Ww, S, w, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0, dev(lo.ravel(), torch.int32), dev(hi.ravel(), torch.int32),
                     max_width=S + 2 * w, beta=(19, 20))
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    agg, upv = H.aggregate(f, cost, sigma, keep_up=True)
    g = torch.from_numpy(np.random.default_rng(9).normal(size=cost.shape).astype(np.float32)).cuda()
    gc, gw, gs = H.aggregate_backward(f, cost, agg, g, sigma, up=upv)
    F = forest_np(f)
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, tlo, thi, _ = orc.kruskal(Hh, Ww, key, lo, hi, beta=(19, 20))
    ref_f = orc.root_forest(Hh, Ww, in_tree, key, 0)
    check_forest(F, ref_f, Hh * Ww, "HDP forest for the adjoint")
    assert F["info"][2] > 20, "expected a forest of many trees"
    D = dmax + 1
    C = np.nan_to_num(orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64),
                                      dmax, tlo, thi), nan=0.0)
    inside = ~np.isnan(volume_to_pixels(cost.cpu().numpy(), F, D))
    G = np.nan_to_num(volume_to_pixels(g.cpu().numpy().astype(np.float64), F, D), nan=0.0)
    ref = adjoint_reference(orc, ref_f["parent"], ref_f["wgt"], ref_f["order"], sigma, C, G)
    got_c = np.nan_to_num(volume_to_pixels(gc.cpu().numpy().astype(np.float64), F, D), nan=0.0)
    check_adjoint(got_c, gw.cpu().numpy().astype(np.float64), float(gs.cpu()), ref,
                  "HDP forest", inside)


def test_adjoint_multi_pair_batch(H, orc):
    """The adjoint of one batched call over pairs of different sizes and label
    ranges (rows padded to the widest range) against per-pair oracle adjoints;
    dsigma is the sum over the batch."""
    shapes = [(40, 56, 7), (33, 47, 15), (24, 64, 3)]
    sigma = 0.1
    pairs = [scenes.small_scene(120 + i, h, w, d) for i, (h, w, d) in enumerate(shapes)]
    lp = H.pyramid(rgb_dev(*[p.left for p in pairs]), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(*[p.right for p in pairs]), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost = H.cost_volume(lp[0], rp[0], shapes, f)
    agg, upv = H.aggregate(f, cost, sigma, keep_up=True)
    g = torch.from_numpy(np.random.default_rng(10).normal(size=cost.shape).astype(np.float32)).cuda()
    gc, gw, gs = H.aggregate_backward(f, cost, agg, g, sigma, up=upv)
    F = forest_np(f)
    D = max(d for _, _, d in shapes) + 1
    gcp = volume_to_pixels(gc.cpu().numpy().astype(np.float64), F, D)
    gp = volume_to_pixels(g.cpu().numpy().astype(np.float64), F, D)
    gwn = gw.cpu().numpy().astype(np.float64)
    off, ds_sum, bs_sum = 0, 0.0, 0.0
    for p, (h, w, d) in zip(pairs, shapes):
        n = h * w
        key = orc.edge_keys(p.left.astype(np.float64), 0)
        in_tree, _, _, _ = orc.kruskal(h, w, key)
        rf = orc.root_forest(h, w, in_tree, key, 0)
        par_g = F["parent"][off:off + n]
        np.testing.assert_array_equal(np.where(par_g >= 0, par_g - off, -1), rf["parent"])
        C = orc.cost_volume(p.left.astype(np.float64), p.right.astype(np.float64), d)
        G = gp[off:off + n, :d + 1]
        ref = adjoint_reference(orc, rf["parent"], rf["wgt"], rf["order"], sigma, C, G)
        ref_pair = dict(ref, ds=0.0, bs=1.0)
        check_adjoint(gcp[off:off + n, :d + 1], gwn[off:off + n], 0.0, ref_pair,
                      f"batch pair {h}x{w} d={d}")
        ds_sum += ref["ds"]; bs_sum += ref["bs"]
        off += n
    assert abs(float(gs.cpu()) - ds_sum) <= REL * bs_sum, (float(gs.cpu()), ds_sum, bs_sum)


def test_graph_replay_matches_eager(H):
    """The whole HDP step captured once and replayed several times (with eager
    work in between) gives the eager result on every replay."""
    shapes = [(96, 128, 63)]
    pair = scenes.small_scene(91, 96, 128, 63)
    L_rgb, R_rgb = rgb_dev(pair.left), rgb_dev(pair.right)
    eager = [r.disp.cpu().numpy() for r in H.hdp_stereo(L_rgb, R_rgb, shapes, S=2, L=2, window=4)]
    step = H.CapturedStep(lambda ws: H.hdp_stereo(L_rgb, R_rgb, shapes, S=2, L=2, window=4, ws=ws))
    for rep in range(4):
        out = step.replay()
        torch.cuda.synchronize()
        for l in range(3):
            np.testing.assert_array_equal(out[l].disp.cpu().numpy(), eager[l],
                                          err_msg=f"replay {rep} layer {l}")
        # unrelated eager work between replays
        H.full_range(R_rgb, L_rgb, [(96, 128, 63)])
        torch.cuda.synchronize()


def test_autograd_tree_aggregate(H, orc):
    """torch.autograd through TreeAggregate gives the oracle's gradients for the
    cost volume, sigma and the per-edge weights; saving or recomputing the
    up-pass checkpoint gives identical gradients."""
    from paper_1509_08197_amd.autograd import tree_aggregate
    Hh, Ww, dmax, sigma = 32, 48, 7, 0.1
    pair = scenes.small_scene(78, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost0 = H.cost_volume(lp[0], rp[0], shapes, f)
    wl = torch.from_numpy(np.random.default_rng(4).normal(size=cost0.shape).astype(np.float32)).cuda()
    grads = []
    for save_up in (True, False):
        cost = cost0.clone().requires_grad_(True)
        sg = torch.tensor(sigma, device="cuda", requires_grad=True)
        wgt = f.array("wgt").clone().requires_grad_(True)
        agg = tree_aggregate(cost, sg, f, wgt, save_up=save_up)
        (agg * wl).sum().backward()
        grads.append((cost.grad.cpu().numpy(), float(sg.grad.cpu()), wgt.grad.cpu().numpy()))
    np.testing.assert_array_equal(grads[0][0], grads[1][0])
    np.testing.assert_array_equal(grads[0][2], grads[1][2])
    assert grads[0][1] == grads[1][1]
    F = forest_np(f)
    node = F["node"]
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, _, _, _ = orc.kruskal(Hh, Ww, key)
    ref = orc.root_forest(Hh, Ww, in_tree, key, 0)
    par, wg, od = ref["parent"], ref["wgt"], ref["order"]
    C = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax)
    Gp = np.zeros_like(C); Gp[node] = wl.cpu().numpy().astype(np.float64)
    dC, dw, ds = orc.aggregate_backward_twopass(par, wg, od, sigma, C, Gp)
    Aabs, Uabs = orc.aggregate_twopass(par, wg, od, sigma, np.abs(Gp), want_up=True)
    AC, UC = orc.aggregate_twopass(par, wg, od, sigma, C, want_up=True)
    got = np.zeros_like(C); got[node] = grads[0][0]
    assert np.all(np.abs(got - dC) <= REL * Aabs)
    s = np.where(par >= 0, np.exp(-wg / sigma), 0.0)
    pp = np.maximum(par, 0)
    B = np.sum(Uabs * (AC[pp] + s[:, None] * UC) + UC * (Aabs[pp] + s[:, None] * Uabs), axis=1)
    B = np.where(par >= 0, B * s / sigma, 0.0)
    assert np.all(np.abs(grads[0][2] - dw) <= REL * B + 1e-30)
    assert abs(grads[0][1] - ds) <= REL * float(np.sum(B * wg / sigma))


def test_native_plan_matches_binding(H):
    """The C-level batch plan (one HIP graph launch per run) gives the labels of
    the Python-orchestrated loop on every layer, for two different inputs."""
    shapes = [(70, 90, 63), (41, 57, 31)]
    plan = H.Plan(shapes, S=2, L=2, window=4)
    for seed in (0, 1):
        pairs = [scenes.small_scene(300 + 10 * seed + i, h, w, d) for i, (h, w, d) in enumerate(shapes)]
        L_rgb = rgb_dev(*[p.left for p in pairs]); R_rgb = rgb_dev(*[p.right for p in pairs])
        ref = H.hdp_stereo(L_rgb, R_rgb, shapes, S=2, L=2, window=4)
        disp = torch.empty(sum(h * w for h, w, _ in shapes), dtype=torch.int32, device="cuda")
        plan.run(L_rgb, R_rgb, disp)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(disp.cpu().numpy(), ref[0].disp.cpu().numpy())
        for l in (1, 2):
            np.testing.assert_array_equal(plan.layer_disp(l).cpu().numpy(),
                                          ref[l].disp.cpu().numpy())
    plan.close()


def test_autograd_interleaved_calls_keep_their_weights(H, orc):
    """Two tree_aggregate calls on one forest with different edge weights, both
    forwards before either backward: each call's gradients are those of its own
    weights, and the forest keeps its own weights afterwards."""
    from paper_1509_08197_amd.autograd import tree_aggregate
    Hh, Ww, dmax, sigma = 24, 40, 5, 0.1
    pair = scenes.small_scene(79, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rp = H.pyramid(rgb_dev(pair.right), shapes, 2, 0)
    f = H.build_tree(lp[0], shapes, 0)
    cost0 = H.cost_volume(lp[0], rp[0], shapes, f)
    own = f.array("wgt").clone()
    rng = np.random.default_rng(12)
    w1 = own * torch.from_numpy(rng.uniform(0.5, 1.5, size=own.shape).astype(np.float32)).cuda()
    w2 = own * torch.from_numpy(rng.uniform(0.5, 1.5, size=own.shape).astype(np.float32)).cuda()
    wl = torch.from_numpy(rng.normal(size=cost0.shape).astype(np.float32)).cuda()
    leaves, outs = [], []
    for wv in (w1, w2):
        c = cost0.clone().requires_grad_(True)
        wt = wv.clone().requires_grad_(True)
        outs.append(tree_aggregate(c, sigma, f, wt))
        leaves.append((c, wt))
    assert torch.equal(f.array("wgt"), own), "forward left other weights in the forest"
    for o in outs:
        (o * wl).sum().backward()
    assert torch.equal(f.array("wgt"), own), "backward left other weights in the forest"
    F = forest_np(f)
    node = F["node"]
    key = orc.edge_keys(pair.left.astype(np.float64), 0)
    in_tree, _, _, _ = orc.kruskal(Hh, Ww, key)
    ref_f = orc.root_forest(Hh, Ww, in_tree, key, 0)
    C = orc.cost_volume(pair.left.astype(np.float64), pair.right.astype(np.float64), dmax)
    G = np.zeros_like(C); G[node] = wl.cpu().numpy().astype(np.float64)
    for k, (wv, (c, wt)) in enumerate(zip((w1, w2), leaves)):
        wg = wv.cpu().numpy().astype(np.float64)
        ref = adjoint_reference(orc, ref_f["parent"], np.where(ref_f["parent"] >= 0, wg, 0.0),
                                ref_f["order"], sigma, C, G)
        got_c = np.zeros_like(C); got_c[node] = c.grad.cpu().numpy()
        check_adjoint(got_c, wt.grad.cpu().numpy().astype(np.float64), ref["ds"], ref,
                      f"interleaved call {k}")


def test_interval_bound_violation_is_reported(H):
    """Pixel intervals that break the bound given to hdp_build_tree (wider than
    max_width, or reaching outside [0, dmax]) are counted, clamped, and turn the
    forest's info read into HDP_EREGIME; the layer still runs inside its buffers."""
    Hh, Ww, dmax = 16, 24, 31
    pair = scenes.small_scene(5, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp, rp = H.pyramid_views(rgb_dev(pair.left), rgb_dev(pair.right), shapes, 2, 0)
    lo = np.full(Hh * Ww, 4, np.int32); hi = np.full(Hh * Ww, 13, np.int32)
    lo[7], hi[7] = 2, 17       # 16 labels > max_width 10
    lo[40], hi[40] = -3, 5     # below label 0
    hi[41] = 40                # above dmax
    f = H.build_tree(lp[0], shapes, 0, dev(lo), dev(hi), max_width=10, beta=(19, 20))
    agg, disp = H.match_layer(lp[0], rp[0], shapes, f)
    torch.cuda.synchronize()
    with pytest.raises(H.HdpError) as e:
        f.read_info()
    assert e.value.code == -4 and f.info[6] == 3
    flo, fhi = f.array("lo").cpu().numpy(), f.array("hi").cpu().numpy()
    assert np.all(flo >= 0) and np.all(fhi <= dmax) and np.all(fhi - flo + 1 <= 10)
    d = disp.cpu().numpy()
    assert np.all((d >= flo) & (d <= fhi))


# --- random spanning tree RT (Section 4.1) -------------------------------------------

def rank_np(seed, n):
    return np.random.default_rng(seed).integers(0, 2 ** 31 - 1, 2 * n).astype(np.int32)


def rt_reference(orc, img, Hh, Ww, level, rank, lo=None, hi=None, beta=(19, 20)):
    """Oracle RT (or HDP+RT forest): Kruskal in (rank, id) order, colour weights."""
    key = orc.edge_keys(img.astype(np.float64), level)
    okey = np.where(key >= 0, rank.astype(np.int64), -1)
    in_tree, tlo, thi, _ = orc.kruskal(Hh, Ww, okey, lo, hi, beta=beta)
    return orc.root_forest(Hh, Ww, in_tree, key, level), tlo, thi


@pytest.mark.parametrize("Hh,Ww,seed", [(120, 160, 1), (31, 47, 2), (1, 64, 3), (64, 1, 4),
                                        (1, 1, 5), (2, 2, 6), (200, 300, 7)])
def test_rt_bit_exact(H, orc, Hh, Ww, seed):
    pair = scenes.small_scene(seed, Hh, Ww, 15)
    shapes = [(Hh, Ww, 15)]
    lv = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    rank = rank_np(seed, Hh * Ww)
    f = H.build_tree(lv[0], shapes, 0, rank=dev(rank))
    F = forest_np(f)
    ref, _, _ = rt_reference(orc, pair.left, Hh, Ww, 0, rank)
    check_forest(F, ref, Hh * Ww, f"RT {Hh}x{Ww}")
    assert F["info"][2] == 1  # one tree
    # a random tree is not the MST (weights ignored by the order)
    if Hh * Ww > 100:
        m = H.build_tree(lv[0], shapes, 0)
        assert not np.array_equal(forest_np(m)["parent"], F["parent"])


@pytest.mark.parametrize("level", [1, 2])
def test_rt_upper_levels_bit_exact(H, orc, level):
    pair = scenes.small_scene(13, 97, 131, 31)
    lv = H.pyramid(rgb_dev(pair.left), [(97, 131, 31)], 2, 2)
    shp = H.level_shapes([(97, 131, 31)], 2, 2)[level]
    n = shp[0][0] * shp[0][1]
    rank = rank_np(50 + level, n)
    f = H.build_tree(lv[level], shp, level, rank=dev(rank))
    F = forest_np(f)
    img = orc.pyramid(pair.left, 2, 2)[level]
    ref, _, _ = rt_reference(orc, img, shp[0][0], shp[0][1], level, rank)
    check_forest(F, ref, n, f"RT level {level}")


def test_hdp_rt_forest_literal_outside_regime(H, orc):
    """HDP+RT outside the exact regime (beta = 3/5): the sequential process in
    the shuffled (rank, id) order, bit-exact against the oracle's."""
    Hh, Ww, dmax, S, w = 48, 64, 63, 2, 4
    pair = scenes.small_scene(66, Hh, Ww, dmax)
    up = np.random.default_rng(5).integers(0, dmax // 2 + 1, ((Hh + 1) // 2, (Ww + 1) // 2))
    up = np.kron(up[::3, ::3], np.ones((3, 3), int))[:up.shape[0], :up.shape[1]]
    lo, hi = orc.predict_range(up, Hh, Ww, S, w, dmax)
    lv = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, dmax)], 2, 0)
    rank = rank_np(77, Hh * Ww)
    f = H.build_tree(lv[0], [(Hh, Ww, dmax)], 0, dev(lo.ravel(), torch.int32),
                     dev(hi.ravel(), torch.int32), max_width=S + 2 * w, beta=(3, 5),
                     rank=dev(rank))
    F = forest_np(f)
    ref, tlo, thi = rt_reference(orc, pair.left, Hh, Ww, 0, rank, lo, hi, beta=(3, 5))
    check_forest(F, ref, Hh * Ww, "literal HDP+RT forest")
    np.testing.assert_array_equal(F["lo"], tlo)
    np.testing.assert_array_equal(F["hi"], thi)
    assert F["info"][6] == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_hdp_rt_forest_bit_exact(H, orc, seed):
    """HDP+RT: the DT rules over the shuffled order, in the exact regime."""
    Hh, Ww, dmax, S, w = 96, 128, 63, 2, 4
    pair = scenes.small_scene(60 + seed, Hh, Ww, dmax)
    up = np.random.default_rng(seed).integers(0, dmax // 2 + 1, ((Hh + 1) // 2, (Ww + 1) // 2))
    up = np.kron(up[::4, ::4], np.ones((4, 4), int))[:up.shape[0], :up.shape[1]]
    lo, hi = orc.predict_range(up, Hh, Ww, S, w, dmax)
    lv = H.pyramid(rgb_dev(pair.left), [(Hh, Ww, dmax)], 2, 0)
    rank = rank_np(70 + seed, Hh * Ww)
    f = H.build_tree(lv[0], [(Hh, Ww, dmax)], 0, dev(lo.ravel(), torch.int32),
                     dev(hi.ravel(), torch.int32), max_width=S + 2 * w, beta=(19, 20),
                     rank=dev(rank))
    F = forest_np(f)
    ref, tlo, thi = rt_reference(orc, pair.left, Hh, Ww, 0, rank, lo, hi)
    check_forest(F, ref, Hh * Ww, "HDP+RT forest")
    np.testing.assert_array_equal(F["lo"], tlo)
    np.testing.assert_array_equal(F["hi"], thi)


def ruler_path_ranks(n_tiles, rng):
    """Edge ranks of a 2 x (32 n_tiles) image whose 32 x 2 tiles form a path:
    edges inside a tile rank 0 (each tile becomes one component in the
    tile-local phase) and the two edges crossing from tile t to t + 1 rank
    2 (1 + v2(t + 1)) plus a random bit, so that every spanning-forest round
    merges the components in pairs only: log2(n_tiles) + 1 hooking rounds."""
    W = 32 * n_tiles
    rank = np.zeros((2, W, 2), np.int64)  # [y, x, dir]: dir 0 joins x + 1, dir 1 joins y + 1
    t = np.arange(n_tiles - 1)
    v2 = np.array([(int(k) & -int(k)).bit_length() - 1 for k in t + 1])
    for y in range(2):
        rank[y, 32 * t + 31, 0] = 2 * (1 + v2) + rng.integers(0, 2, n_tiles - 1)
    return rank.reshape(-1).astype(np.int32)


@pytest.mark.parametrize("n_pairs,tail_mode", [(2, "lds"), (8, "global")])
def test_rt_ruler_path_many_rounds(H, orc, n_pairs, tail_mode):
    """Spanning-forest rounds past the full-grid and compacted-list rounds: a
    batch of 2 x 262144 pairs of 8192 tiles each needs 13 hooking rounds, so
    the one-workgroup tail finishes the last one, in LDS (2 pairs: 2044 live
    edges after the full-grid rounds) or in global memory (8 pairs: 8176).
    Every pair's tree against the oracle's Kruskal in (rank, id) order."""
    n_tiles, Hh = 8192, 2
    Ww = 32 * n_tiles
    rng = np.random.default_rng(40 + n_pairs)
    imgs = [rng.integers(0, 256, (Hh, Ww, 3), dtype=np.uint8) for _ in range(n_pairs)]
    ranks = [ruler_path_ranks(n_tiles, rng) for _ in range(n_pairs)]
    shapes = [(Hh, Ww, 15)] * n_pairs
    lv = H.pyramid(rgb_dev(*imgs), shapes, 2, 0)
    f = H.build_tree(lv[0], shapes, 0, rank=dev(np.concatenate(ranks)))
    F = forest_np(f)
    info = F["info"]
    assert info[H.INFO["error"]] == 0
    assert info[H.INFO["n_trees"]] == n_pairs
    assert info[H.INFO["mst_rounds"]] == 13, info[H.INFO["mst_rounds"]]
    assert info[H.INFO["live_edges"]] == n_pairs * 2 * (n_tiles - 1)
    assert info[H.INFO["list_edges"]] == n_pairs * 2 * (n_tiles // 16 - 1)
    assert (info[H.INFO["list_edges"]] > 6144) == (tail_mode == "global")
    n = Hh * Ww
    for i in range(n_pairs):
        ref, _, _ = rt_reference(orc, imgs[i], Hh, Ww, 0, ranks[i])
        par = F["parent"][i * n:(i + 1) * n]
        np.testing.assert_array_equal(np.where(par >= 0, par - i * n, -1), ref["parent"],
                                      err_msg=f"pair {i} parent")
        np.testing.assert_array_equal(F["depth"][i * n:(i + 1) * n], ref["depth"],
                                      err_msg=f"pair {i} depth")


def test_hdp_rt_loop_stagewise(H, orc):
    """The whole HDP+RT loop: every layer's forest and aggregation against the
    oracle's loop with the same ranks (layer l fed the oracle's layer l+1
    labels), and the fused matching equal to the three separate steps."""
    Hh, Ww, dmax, S, w, L = 96, 128, 63, 2, 4, 3
    pair = scenes.small_scene(90, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lvs = H.level_shapes(shapes, S, L)
    ranks = [rank_np(900 + l, lvs[l][0][0] * lvs[l][0][1]) for l in range(L + 1)]
    ores = orc.hdp_stereo(pair.left, pair.right, dmax, S=S, L=L, window=w, want_forest=True,
                          ranks=[r.astype(np.int64) for r in ranks])
    lp = H.pyramid(rgb_dev(pair.left), shapes, S, L)
    rp = H.pyramid(rgb_dev(pair.right), shapes, S, L)
    for level in range(L, -1, -1):
        dl = lvs[level][0][2]
        lo = hi = None
        if level < L:
            up = dev(ores[level + 1]["disp"].ravel(), torch.int32)
            lo, hi = H.predict_range(up, lvs[level + 1], lvs[level], S, w)
        r = H.stereo_level(lp[level], rp[level], lvs[level], level, lo, hi,
                           max_width=min(S + 2 * w, dl + 1), keep=True, rank=dev(ranks[level]))
        F = forest_np(r.forest)
        assert F["info"][7] == 0
        np.testing.assert_array_equal(F["parent"], ores[level]["parent"])
        np.testing.assert_array_equal(F["lo"], ores[level]["tree_lo"])
        np.testing.assert_array_equal(F["hi"], ores[level]["tree_hi"])
        Lf = orc.pyramid(pair.left, S, L)[level]; Rf = orc.pyramid(pair.right, S, L)[level]
        ref, tlo, thi = rt_reference(orc, Lf, lvs[level][0][0], lvs[level][0][1], level,
                                     ranks[level],
                                     None if lo is None else ores[level]["pix_lo"],
                                     None if lo is None else ores[level]["pix_hi"])
        if lo is None:
            tlo = np.zeros(F["lo"].shape, np.int32); thi = np.full(F["hi"].shape, dl, np.int32)
        cost = orc.cost_volume(Lf, Rf, dl, tlo, thi)
        agg = orc.aggregate_twopass(ref["parent"], ref["wgt"], ref["order"], 0.1,
                                    np.nan_to_num(cost, nan=0.0))
        agg[np.isnan(cost)] = np.nan
        assert_rel(volume_to_pixels(r.agg.cpu().numpy(), F, dl + 1), agg, REL,
                   f"HDP+RT aggregate layer {level}")
        nm, nt = check_wta(r.disp.cpu().numpy(), agg, tlo, thi, f"HDP+RT WTA layer {level}")
        fused = H.stereo_level(lp[level], rp[level], lvs[level], level, lo, hi,
                               max_width=min(S + 2 * w, dl + 1), rank=dev(ranks[level]))
        assert torch.equal(fused.disp, r.disp), f"layer {level}: fused labels differ"
        print(f"HDP+RT layer {level}: WTA mismatches {nm} (near-ties {nt})")


# --- Bayesian interval prediction (Section 2.2 eq. dpm, Section 3.1 eq. crtr) -------

GMM_LOW = [(50, 70, 255), (33, 41, 191), (17, 9, 63), (5, 6, 1)]


def gmm_case(seed):
    rng = np.random.default_rng(seed)
    K = 1 + seed % 4
    pi = rng.dirichlet(np.ones(K)); mu = rng.uniform(-1.5, 1.5, K); sd = rng.uniform(0.3, 2.0, K)
    prior = np.zeros((len(GMM_LOW), 256))
    for p, (_, _, d) in enumerate(GMM_LOW):
        prior[p, :d + 1] = rng.integers(0, 4, d + 1) * (rng.random(d + 1) < 0.6)
    prior[2, :] = 0.0  # a pair without prior mass: the model alone
    return pi, mu, sd, prior


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_interval_table_bit_exact(H, orc, seed):
    S = 2
    upper = [((h + 1) // 2, (w + 1) // 2, d // 2) for h, w, d in GMM_LOW]
    pi, mu, sd, prior = gmm_case(seed)
    g = H.make_gmm(pi, mu, sd)
    for delta in (0.004, 0.016, 0.2, 1.0):
        lo_t, hi_t, mw = H.interval_table(upper, GMM_LOW, S, g, dev(prior), delta)
        lo_t, hi_t = lo_t.cpu().numpy(), hi_t.cpu().numpy()
        widest = 0
        for p, (_, _, d) in enumerate(GMM_LOW):
            olo, ohi = orc.gmm_interval_table(S, d, d // 2, pi, mu, sd, prior[p, :d + 1], delta)
            np.testing.assert_array_equal(lo_t[p, :d // 2 + 1], olo, err_msg=f"pair {p} {delta}")
            np.testing.assert_array_equal(hi_t[p, :d // 2 + 1], ohi, err_msg=f"pair {p} {delta}")
            widest = max(widest, int((ohi - olo + 1).max()))
        assert int(mw.item()) == widest
        if delta == 1.0:  # nothing passes eq. crtr: single labels
            for p, (_, _, d) in enumerate(GMM_LOW):
                assert (lo_t[p, :d // 2 + 1] == hi_t[p, :d // 2 + 1]).all()


def test_interval_table_degenerate_models(H, orc):
    """A model that underflows everywhere gives the child blocks; a sharp model
    at offset 0 with a flat prior gives them too."""
    S = 2
    upper = [((h + 1) // 2, (w + 1) // 2, d // 2) for h, w, d in GMM_LOW]
    prior = np.ones((len(GMM_LOW), 256))
    for mu, sd in ((500.0, 0.01), (0.0, 0.05)):
        lo_t, hi_t, _ = H.interval_table(upper, GMM_LOW, S, H.make_gmm([1.0], [mu], [sd]),
                                         dev(prior), 0.01)
        for p, (_, _, d) in enumerate(GMM_LOW):
            i = np.arange(d // 2 + 1)
            np.testing.assert_array_equal(lo_t[p, :d // 2 + 1].cpu().numpy(), np.minimum(2 * i, d))
            np.testing.assert_array_equal(hi_t[p, :d // 2 + 1].cpu().numpy(),
                                          np.minimum(2 * i + 1, d))


def test_predict_range_table_bit_exact(H, orc):
    S = 2
    upper = [((h + 1) // 2, (w + 1) // 2, d // 2) for h, w, d in GMM_LOW]
    pi, mu, sd, prior = gmm_case(5)
    lo_t, hi_t, _ = H.interval_table(upper, GMM_LOW, S, H.make_gmm(pi, mu, sd), dev(prior), 0.004)
    rng = np.random.default_rng(6)
    ups = [rng.integers(0, d + 1, (h, w)).astype(np.int32) for h, w, d in upper]
    up = dev(np.concatenate([u.ravel() for u in ups]))
    lo, hi = H.predict_range_table(up, upper, GMM_LOW, S, lo_t, hi_t)
    lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
    off = 0
    for p, (h, w, d) in enumerate(GMM_LOW):
        olo, ohi = orc.predict_range_table(ups[p], h, w, S, lo_t[p].cpu().numpy(),
                                           hi_t[p].cpu().numpy())
        np.testing.assert_array_equal(lo[off:off + h * w], olo.ravel())
        np.testing.assert_array_equal(hi[off:off + h * w], ohi.ravel())
        off += h * w


def test_hdp_gmm_loop_stagewise(H, orc):
    """The HDP loop with Bayesian intervals: every layer fed the oracle's
    layer-(l+1) labels gives the oracle's table, pixel intervals, disparity
    forest and aggregation; the GPU loop then runs end to end."""
    Hh, Ww, dmax, S, L = 96, 128, 63, 2, 3
    pair = scenes.small_scene(77, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lvs = H.level_shapes(shapes, S, L)
    gm = scenes.gmm_params(3, L)
    priors = [scenes.label_prior(pair.gt, S, l, lvs[l][0][2]) for l in range(L)]
    delta0 = 0.004
    lp = H.pyramid(rgb_dev(pair.left), shapes, S, L)
    rp = H.pyramid(rgb_dev(pair.right), shapes, S, L)
    Lf = orc.pyramid(pair.left, S, L); Rf = orc.pyramid(pair.right, S, L)
    o_up = orc.stereo_level(Lf[L], Rf[L], lvs[L][0][2], L)
    for level in range(L - 1, -1, -1):
        dl = lvs[level][0][2]
        Hl, Wl = lvs[level][0][:2]
        olo_t, ohi_t = orc.gmm_interval_table(S, dl, lvs[level + 1][0][2], *gm[level],
                                              priors[level], delta0 * S ** level)
        olo, ohi = orc.predict_range_table(o_up["disp"], Hl, Wl, S, olo_t, ohi_t)
        lo_t, hi_t, mw = H.interval_table(lvs[level + 1], lvs[level], S, H.make_gmm(*gm[level]),
                                          dev(priors[level][None, :]), delta0 * S ** level)
        np.testing.assert_array_equal(lo_t[0].cpu().numpy(), olo_t)
        np.testing.assert_array_equal(hi_t[0].cpu().numpy(), ohi_t)
        up = dev(o_up["disp"].ravel(), torch.int32)
        lo, hi = H.predict_range_table(up, lvs[level + 1], lvs[level], S, lo_t, hi_t)
        np.testing.assert_array_equal(lo.cpu().numpy(), olo.ravel())
        np.testing.assert_array_equal(hi.cpu().numpy(), ohi.ravel())
        mwi = int(mw.item())
        assert 19 * mwi > 20 * (mwi - 1), "test case left the exact regime"
        r = H.stereo_level(lp[level], rp[level], lvs[level], level, lo, hi, max_width=mwi,
                           keep=True)
        o = orc.stereo_level(Lf[level], Rf[level], dl, level, olo, ohi)
        F = forest_np(r.forest)
        assert F["info"][7] == 0 and F["info"][6] == 0
        np.testing.assert_array_equal(F["parent"], o["parent"])
        np.testing.assert_array_equal(F["lo"], o["tree_lo"])
        np.testing.assert_array_equal(F["hi"], o["tree_hi"])
        ref = run_level_oracle(orc, Lf[level], Rf[level], dl, level, olo, ohi)
        assert_rel(volume_to_pixels(r.agg.cpu().numpy(), F, dl + 1), ref["agg"], REL,
                   f"GMM aggregate layer {level}")
        nm, nt = check_wta(r.disp.cpu().numpy(), ref["agg"], ref["tlo"], ref["thi"],
                           f"GMM WTA layer {level}")
        print(f"GMM layer {level}: widest interval {mwi}, WTA mismatches {nm} (near-ties {nt})")
        o_up = o
    # the whole loop on the GPU with these models runs and labels every pixel
    res = H.hdp_stereo(rgb_dev(pair.left), rgb_dev(pair.right), shapes, S=S, L=L,
                       gmm=[H.make_gmm(*g) for g in gm],
                       priors=[dev(p[None, :]) for p in priors], delta0=delta0)
    d0 = res[0].disp.cpu().numpy()
    assert d0.min() >= 0 and d0.max() <= dmax


def test_hdp_gmm_layers_literal_forest(H, orc):
    """Bayesian intervals with beta = 3/5 (outside the exact regime): every
    layer fed the oracle's layer-(l+1) labels gives the oracle's literal
    disparity forest (parents and tree intervals bit for bit), aggregation
    (within 1e-5) and labels (up to near-ties)."""
    Hh, Ww, dmax, S, L = 64, 80, 63, 2, 2
    beta = (3, 5)
    pair = scenes.small_scene(79, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lvs = H.level_shapes(shapes, S, L)
    gm = scenes.gmm_params(3, L)
    priors = [scenes.label_prior(pair.gt, S, l, lvs[l][0][2]) for l in range(L)]
    delta0 = 0.004
    lp = H.pyramid(rgb_dev(pair.left), shapes, S, L)
    rp = H.pyramid(rgb_dev(pair.right), shapes, S, L)
    Lf = orc.pyramid(pair.left, S, L); Rf = orc.pyramid(pair.right, S, L)
    o_up = orc.stereo_level(Lf[L], Rf[L], lvs[L][0][2], L)
    for level in range(L - 1, -1, -1):
        dl = lvs[level][0][2]
        Hl, Wl = lvs[level][0][:2]
        olo_t, ohi_t = orc.gmm_interval_table(S, dl, lvs[level + 1][0][2], *gm[level],
                                              priors[level], delta0 * S ** level)
        olo, ohi = orc.predict_range_table(o_up["disp"], Hl, Wl, S, olo_t, ohi_t)
        lo_t, hi_t, mw = H.interval_table(lvs[level + 1], lvs[level], S, H.make_gmm(*gm[level]),
                                          dev(priors[level][None, :]), delta0 * S ** level)
        up = dev(o_up["disp"].ravel(), torch.int32)
        lo, hi = H.predict_range_table(up, lvs[level + 1], lvs[level], S, lo_t, hi_t)
        mwi = int(mw.item())
        assert beta[0] * mwi <= beta[1] * (mwi - 1), "test case is inside the exact regime"
        r = H.stereo_level(lp[level], rp[level], lvs[level], level, lo, hi, max_width=mwi,
                           beta=beta, keep=True)
        o = orc.stereo_level(Lf[level], Rf[level], dl, level, olo, ohi, beta=beta)
        F = forest_np(r.forest)
        assert F["info"][7] == 0 and F["info"][6] == 0
        np.testing.assert_array_equal(F["parent"], o["parent"])
        np.testing.assert_array_equal(F["lo"], o["tree_lo"])
        np.testing.assert_array_equal(F["hi"], o["tree_hi"])
        key = orc.edge_keys(Lf[level], level)
        in_tree, tlo, thi, _ = orc.kruskal(Hl, Wl, key, olo, ohi, beta=beta)
        ref_f = orc.root_forest(Hl, Wl, in_tree, key, level)
        cost = orc.cost_volume(Lf[level], Rf[level], dl, tlo, thi)
        agg = orc.aggregate_twopass(ref_f["parent"], ref_f["wgt"], ref_f["order"], 0.1,
                                    np.nan_to_num(cost, nan=0.0))
        agg[np.isnan(cost)] = np.nan
        assert_rel(volume_to_pixels(r.agg.cpu().numpy(), F, dl + 1), agg, REL,
                   f"literal GMM aggregate layer {level}")
        nm, nt = check_wta(r.disp.cpu().numpy(), agg, tlo, thi, f"literal GMM WTA layer {level}")
        print(f"literal GMM layer {level}: widest pixel interval {mwi}, widest tree interval "
              f"{int((F['hi'] - F['lo']).max()) + 1}, WTA mismatches {nm} (near-ties {nt})")
        o_up = o


# --- left-right check, sampled prior, refinement (Sections 3.1, 3.3) ----------------

LR_SHAPES = [(37, 53, 31), (20, 9, 7), (1, 1, 3), (64, 96, 63)]


def test_mirror_and_lr_check_bit_exact(H, orc):
    rng = np.random.default_rng(8)
    imgs = [rng.integers(0, 256, (h, w, 3)).astype(np.uint8) for h, w, _ in LR_SHAPES]
    m = H.mirror(rgb_dev(*imgs), LR_SHAPES).cpu().numpy()
    off = 0
    for im, (h, w, _) in zip(imgs, LR_SHAPES):
        np.testing.assert_array_equal(m[off:off + h * w].reshape(h, w, 3), im[:, ::-1])
        off += h * w
    dls = [rng.integers(0, d + 1, (h, w)).astype(np.int32) for h, w, d in LR_SHAPES]
    # right labels equal to the left ones at the match for about half the pixels
    drs = []
    for dl, (h, w, d) in zip(dls, LR_SHAPES):
        dr = rng.integers(0, d + 1, (h, w)).astype(np.int32)
        for y in range(h):
            for x in range(w):
                if x - dl[y, x] >= 0 and rng.random() < 0.5:
                    dr[y, x - dl[y, x]] = dl[y, x]
        drs.append(dr)
    cat = lambda a: dev(np.concatenate([x.ravel() for x in a]))
    for tol in (0, 1):
        st_m = H.lr_check(cat(dls), cat([d[:, ::-1] for d in drs]), LR_SHAPES, tol).cpu().numpy()
        st_n = H.lr_check(cat(dls), cat(drs), LR_SHAPES, tol, right_mirrored=False).cpu().numpy()
        np.testing.assert_array_equal(st_m, st_n)
        off = 0
        for dl, dr, (h, w, _) in zip(dls, drs, LR_SHAPES):
            ref = orc.lr_check(dl, np.ascontiguousarray(dr[:, ::-1]), tol)
            np.testing.assert_array_equal(st_m[off:off + h * w], ref.ravel())
            off += h * w


def test_sample_prior_bit_exact(H, orc):
    rng = np.random.default_rng(9)
    dls = [rng.integers(0, d + 1, (h, w)).astype(np.int32) for h, w, d in LR_SHAPES]
    sts = [(rng.random((h, w)) < 0.7).astype(np.uint8) for h, w, _ in LR_SHAPES]
    cat = lambda a: dev(np.concatenate([x.ravel() for x in a]))
    for square in (5, 3):
        pr = H.sample_prior(cat(dls), cat(sts), LR_SHAPES, square, stride=70).cpu().numpy()
        for p, (dl, s, (h, w, d)) in enumerate(zip(dls, sts, LR_SHAPES)):
            ref = orc.sample_prior(dl, s, d, square)
            np.testing.assert_array_equal(pr[p, :d + 1], ref)
            assert (pr[p, d + 1:] == 0).all()


@pytest.mark.parametrize("hdp_layer", [False, True])
def test_refine_matches_oracle(H, orc, hdp_layer):
    """Refinement over a layer's forest with the oracle's labels and stable
    pixels as input: aggregated refinement cost within 1e-5 of FP64, labels
    equal except at near-ties."""
    Hh, Ww, dmax = 72, 96, 31
    pair = scenes.small_scene(33, Hh, Ww, dmax)
    shapes = [(Hh, Ww, dmax)]
    lp = H.pyramid(rgb_dev(pair.left), shapes, 2, 0)
    Lf = pair.left.astype(np.float64)
    lo = hi = None
    kw = {}
    if hdp_layer:
        up = np.random.default_rng(2).integers(0, dmax // 2 + 1, (Hh // 2, Ww // 2))
        up = np.kron(up[::4, ::4], np.ones((4, 4), int))[:Hh // 2, :Ww // 2]
        lo, hi = orc.predict_range(up, Hh, Ww, 2, 4, dmax)
        kw = dict(pix_lo=dev(lo.ravel(), torch.int32), pix_hi=dev(hi.ravel(), torch.int32),
                  max_width=10)
    f = H.build_tree(lp[0], shapes, 0, **kw)
    ref = run_level_oracle(orc, Lf, pair.right.astype(np.float64), dmax, 0, lo, hi)
    rng = np.random.default_rng(4)
    disp = np.clip(np.rint(pair.gt).astype(np.int32), 0, dmax)
    if hdp_layer:
        disp = np.clip(disp, ref["tlo"].reshape(Hh, Ww), ref["thi"].reshape(Hh, Ww))
    stable = (rng.random((Hh, Ww)) < 0.6).astype(np.uint8)
    agg, lab = H.refine(f, dev(disp.ravel()), dev(stable.ravel()))
    F = forest_np(f)
    cost = orc.refine_cost(disp, stable, dmax, ref["tlo"], ref["thi"])
    oagg = orc.aggregate_twopass(ref["ref"]["parent"], ref["ref"]["wgt"], ref["ref"]["order"],
                                 0.1, np.nan_to_num(cost, nan=0.0))
    oagg[np.isnan(cost)] = np.nan
    got = volume_to_pixels(agg.cpu().numpy(), F, dmax + 1)
    # entries whose exact value is 0 (no stable pixel contributes) must be 0
    zero = oagg == 0
    assert (got[zero] == 0).all()
    assert_rel(got[~zero], oagg[~zero], REL, "refinement aggregate")
    nm, nt = check_wta(lab.cpu().numpy(), oagg, ref["tlo"], ref["thi"], "refinement WTA")
    print(f"refinement ({'HDP' if hdp_layer else 'MST'}): mismatches {nm} (near-ties {nt})")


def test_right_view_and_check_end_to_end(H, orc):
    """Left run, run on the mirrored pair and the check on the GPU, against the
    same chain in the oracle: labels equal except at near-ties, and the stable
    mask equal wherever both views' labels agree with the oracle's."""
    pair = scenes.workload(1)
    Hh, Ww = pair.shape
    shapes = [(Hh, Ww, pair.dmax)]
    L8, R8 = rgb_dev(pair.left), rgb_dev(pair.right)
    left = H.full_range(L8, R8, shapes)
    right = H.full_range(H.mirror(R8, shapes), H.mirror(L8, shapes), shapes)
    st = H.lr_check(left.disp, right.disp, shapes).cpu().numpy()
    fl, fr = pair.left.astype(np.float64), pair.right.astype(np.float64)
    ol = orc.stereo_level(fl, fr, pair.dmax, 0)
    orr = orc.stereo_level(orc.mirrored(fr), orc.mirrored(fl), pair.dmax, 0)
    ost = orc.lr_check(ol["disp"], orr["disp"], 0).ravel()
    gl, gr = left.disp.cpu().numpy(), right.disp.cpu().numpy()
    for g, o, what in ((gl, ol, "left"), (gr, orr, "mirrored right")):
        mism = g != o["disp"].ravel()
        near = (o["c2"] - o["c1"]) <= REL * np.abs(o["c1"])
        assert np.all(near[mism]), f"{what}: mismatches off near-ties"
    same = (gl == ol["disp"].ravel()) & (gr == orr["disp"].ravel())
    assert same.mean() > 0.99
    # where both label maps agree everywhere the check reads, the masks agree
    x = np.arange(Hh * Ww) % Ww
    y = np.arange(Hh * Ww) // Ww
    xr = x - gl
    inside = (xr >= 0) & (xr < Ww)
    j = y * Ww + (Ww - 1 - np.clip(xr, 0, Ww - 1))
    ok = same & same[j]
    np.testing.assert_array_equal(st[ok | ~inside], ost[ok | ~inside])
    assert st.mean() > 0.5
