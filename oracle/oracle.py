"""Python front-end of the FP64 CPU oracle (``hdp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the GPU library or its binding.

The C source is compiled with gcc into ``liboracle.so`` next to this file.
Functions mirror the C entry points and take / return numpy arrays.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Default cost constants {a_c, tau_c, a_g, tau_g} (0-255 intensity units).
COST_PARAMS = (0.89, 7.0, 0.11, 2.0)


def _prm(prm):
    """Cost constants (a_c, tau_c, a_g, tau_g[, border]) as the C array; border
    0 (default): a label past the left image border costs both truncations;
    1: it is compared with the row's first pixel."""
    pr = [float(x) for x in prm]
    return np.array(pr + [0.0] * (5 - len(pr)), np.float64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (single-threaded, -O2, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I = C.c_int
D = C.c_double


def _declare(L):
    L.or_level_dims.argtypes = [I, I, I, I, I, P, P, P]
    L.or_pyramid.argtypes = [P, I, I, I, I, P]
    L.or_matching_cost.argtypes = [P, P, I, I, I, I, I, P]
    L.or_matching_cost.restype = D
    L.or_cost_volume.argtypes = [P, P, I, I, I, P, P, P, P]
    L.or_edge_keys.argtypes = [P, I, I, I, P]
    L.or_kruskal.argtypes = [I, I, P, P, P, I, I, P, P, P]
    L.or_kruskal.restype = I
    L.or_root_forest.argtypes = [I, I, P, P, I, P, P, P, P, P, P]
    L.or_root_forest.restype = I
    L.or_aggregate_direct.argtypes = [I, I, P, P, D, I, P, P, I, P]
    L.or_aggregate_twopass.argtypes = [I, P, P, P, D, I, P, P, P]
    L.or_wta.argtypes = [I, I, P, P, P, P, P, P]
    L.or_predict_range.argtypes = [P, I, I, I, I, I, I, I, P, P]
    L.or_gmm_interval_table.argtypes = [I, I, I, I, P, P, P, P, D, P, P]
    L.or_predict_range_table.argtypes = [P, I, I, I, I, I, P, P, P, P]
    L.or_lr_check.argtypes = [P, P, I, I, I, P]
    L.or_sample_prior.argtypes = [P, P, I, I, I, I, P]
    L.or_refine_cost.argtypes = [P, P, I, I, P, P, P]
    L.or_stereo_level.argtypes = [P, P, I, I, I, I, P, P, I, I, D, P,
                                  P, P, P, P, P, P, P, P, P, I, P, P, P]
    L.or_stereo_level.restype = I
    L.or_aggregate_grad_dense.argtypes = [I, I, P, P, D, I, P, P, P, P, P]
    L.or_aggregate_backward_twopass.argtypes = [I, P, P, P, D, I, P, P, P, P, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --- graph pyramid -----------------------------------------------------------

def level_dims(H, W, dmax, S, L):
    Hs = np.zeros(L + 1, np.int32); Ws = np.zeros(L + 1, np.int32); ds = np.zeros(L + 1, np.int32)
    lib().or_level_dims(H, W, dmax, S, L, _p(Hs), _p(Ws), _p(ds))
    return [int(v) for v in Hs], [int(v) for v in Ws], [int(v) for v in ds]


def pyramid(rgb, S, L):
    """List of (H_l, W_l, 3) float64 level images, l = 0..L."""
    rgb = _c(rgb, np.uint8)
    H, W = rgb.shape[:2]
    Hs, Ws, _ = level_dims(H, W, 0, S, L)
    total = sum(h * w * 3 for h, w in zip(Hs, Ws))
    out = np.zeros(total, np.float64)
    lib().or_pyramid(_p(rgb), H, W, S, L, _p(out))
    levels, off = [], 0
    for h, w in zip(Hs, Ws):
        levels.append(out[off:off + h * w * 3].reshape(h, w, 3)); off += h * w * 3
    return levels


# --- matching cost -----------------------------------------------------------

def matching_cost(left, right, x, y, d, prm=COST_PARAMS):
    left = _c(left, np.float64); right = _c(right, np.float64)
    H, W = left.shape[:2]
    pr = _prm(prm)
    return lib().or_matching_cost(_p(left), _p(right), H, W, x, y, d, _p(pr))


def cost_volume(left, right, dmax, lo=None, hi=None, prm=COST_PARAMS):
    """[N][dmax+1] float64, NaN outside [lo, hi]."""
    left = _c(left, np.float64); right = _c(right, np.float64)
    H, W = left.shape[:2]
    out = np.zeros((H * W, dmax + 1), np.float64)
    pr = _prm(prm)
    lo = None if lo is None else _c(lo, np.int32).ravel()
    hi = None if hi is None else _c(hi, np.int32).ravel()
    lib().or_cost_volume(_p(left), _p(right), H, W, dmax, _p(lo), _p(hi), _p(pr), _p(out))
    return out


# --- trees -------------------------------------------------------------------

def edge_keys(img, level):
    img = _c(img, np.float64)
    H, W = img.shape[:2]
    key = np.zeros(2 * H * W, np.int64)
    lib().or_edge_keys(_p(img), H, W, level, _p(key))
    return key


def kruskal(H, W, key, pix_lo=None, pix_hi=None, beta=(19, 20)):
    """Returns (in_tree[2N] uint8, tree_lo, tree_hi, n_edges)."""
    key = _c(key, np.int64)
    N = H * W
    in_tree = np.zeros(2 * N, np.uint8)
    tlo = thi = None
    if pix_lo is not None:
        pix_lo = _c(pix_lo, np.int32).ravel(); pix_hi = _c(pix_hi, np.int32).ravel()
        tlo = np.zeros(N, np.int32); thi = np.zeros(N, np.int32)
    n = lib().or_kruskal(H, W, _p(key), _p(pix_lo), _p(pix_hi), int(beta[0]), int(beta[1]),
                         _p(in_tree), _p(tlo), _p(thi))
    return in_tree, tlo, thi, n


def root_forest(H, W, in_tree, key, level):
    """Returns dict(parent, wgt, depth, tree, order, level_ptr, n_levels)."""
    N = H * W
    in_tree = _c(in_tree, np.uint8); key = _c(key, np.int64)
    parent = np.zeros(N, np.int32); depth = np.zeros(N, np.int32); tree = np.zeros(N, np.int32)
    order = np.zeros(N, np.int32); lptr = np.zeros(N + 1, np.int32); wgt = np.zeros(N, np.float64)
    nl = lib().or_root_forest(H, W, _p(in_tree), _p(key), level, _p(parent), _p(wgt), _p(depth),
                              _p(tree), _p(order), _p(lptr))
    return dict(parent=parent, wgt=wgt, depth=depth, tree=tree, order=order,
                level_ptr=lptr[:nl + 1].copy(), n_levels=nl)


def edge_weights(key, level):
    """Grid-edge weights key / (255 * 4^level); NaN for edges leaving the image."""
    key = np.asarray(key)
    w = key.astype(np.float64) / (255.0 * 4.0 ** level)
    w[key < 0] = np.nan
    return w


# --- aggregation -------------------------------------------------------------

def aggregate_direct(H, W, in_tree, edge_w, sigma, cost, pixels=None):
    cost = _c(cost, np.float64)
    N, Dn = cost.shape
    in_tree = _c(in_tree, np.uint8); edge_w = _c(np.nan_to_num(edge_w, nan=0.0), np.float64)
    pix = np.arange(N, dtype=np.int32) if pixels is None else _c(pixels, np.int32)
    out = np.zeros((len(pix), Dn), np.float64)
    lib().or_aggregate_direct(H, W, _p(in_tree), _p(edge_w), float(sigma), Dn, _p(cost),
                              _p(pix), len(pix), _p(out))
    return out


def aggregate_twopass(parent, wgt, order, sigma, cost, want_up=False):
    cost = _c(cost, np.float64)
    N, Dn = cost.shape
    out = np.zeros_like(cost)
    up = np.zeros_like(cost) if want_up else None
    lib().or_aggregate_twopass(N, _p(_c(parent, np.int32)), _p(_c(wgt, np.float64)),
                               _p(_c(order, np.int32)), float(sigma), Dn, _p(cost), _p(out),
                               _p(up))
    return (out, up) if want_up else out


def wta(agg, lo=None, hi=None):
    agg = _c(agg, np.float64)
    N, Dn = agg.shape
    disp = np.zeros(N, np.int32); c1 = np.zeros(N); c2 = np.zeros(N)
    lo = None if lo is None else _c(lo, np.int32).ravel()
    hi = None if hi is None else _c(hi, np.int32).ravel()
    lib().or_wta(N, Dn, _p(agg), _p(lo), _p(hi), _p(disp), _p(c1), _p(c2))
    return disp, c1, c2


def predict_range(disp_up, H, W, S, window, dmax_l):
    disp_up = _c(disp_up, np.int32)
    Hu, Wu = disp_up.shape
    lo = np.zeros((H, W), np.int32); hi = np.zeros((H, W), np.int32)
    lib().or_predict_range(_p(disp_up), Hu, Wu, H, W, S, window, dmax_l, _p(lo), _p(hi))
    return lo, hi


def gmm_interval_table(S, dl, d_up, pi, mu, sd, prior, delta):
    """Per parent label i = 0..d_up the Bayesian interval (lo, hi) of layer l
    (Section 2.2 eq. dpm, Section 3.1 eq. crtr)."""
    pi = _c(pi, np.float64); mu = _c(mu, np.float64); sd = _c(sd, np.float64)
    prior = _c(prior, np.float64)
    assert len(pi) == len(mu) == len(sd) and len(prior) == dl + 1
    lo = np.zeros(d_up + 1, np.int32); hi = np.zeros(d_up + 1, np.int32)
    lib().or_gmm_interval_table(int(S), int(dl), int(d_up), len(pi), _p(pi), _p(mu), _p(sd),
                                _p(prior), float(delta), _p(lo), _p(hi))
    return lo, hi


def predict_range_table(disp_up, H, W, S, lo_tab, hi_tab):
    disp_up = _c(disp_up, np.int32)
    Hu, Wu = disp_up.shape
    lo = np.zeros((H, W), np.int32); hi = np.zeros((H, W), np.int32)
    lib().or_predict_range_table(_p(disp_up), Hu, Wu, H, W, S, _p(_c(lo_tab, np.int32)),
                                 _p(_c(hi_tab, np.int32)), _p(lo), _p(hi))
    return lo, hi


def lr_check(disp_l, disp_r_mir, tol=0):
    """Stable pixels (uint8 0/1) of the left view given the right view's labels
    in mirrored coordinates (the left-reference output of the mirrored pair)."""
    disp_l = _c(disp_l, np.int32); disp_r_mir = _c(disp_r_mir, np.int32)
    H, W = disp_l.shape
    out = np.zeros((H, W), np.uint8)
    lib().or_lr_check(_p(disp_l), _p(disp_r_mir), H, W, int(tol), _p(out))
    return out


def mirrored(img):
    """The pair's image flipped left to right (the reference for the right view)."""
    return np.ascontiguousarray(np.asarray(img)[:, ::-1])


def sample_prior(disp, stable, dmax, square=5):
    disp = _c(disp, np.int32); stable = _c(stable, np.uint8)
    H, W = disp.shape
    prior = np.zeros(dmax + 1, np.float64)
    lib().or_sample_prior(_p(disp), _p(stable), H, W, int(square), int(dmax), _p(prior))
    return prior


def refine_cost(disp, stable, dmax, lo=None, hi=None):
    disp = _c(disp, np.int32).ravel(); stable = _c(stable, np.uint8).ravel()
    N = disp.size
    cost = np.zeros((N, dmax + 1), np.float64)
    lo = None if lo is None else _c(lo, np.int32).ravel()
    hi = None if hi is None else _c(hi, np.int32).ravel()
    lib().or_refine_cost(_p(disp), _p(stable), N, int(dmax), _p(lo), _p(hi), _p(cost))
    return cost


def refine_level(forest, disp, stable, dmax, sigma=0.1, lo=None, hi=None):
    """Tree-based refinement of one layer's labels over its forest (Section
    3.3 closing paragraph): refinement cost, two-pass aggregation, WTA.
    forest: dict with parent, wgt, order (root_forest / stereo_level output).
    Returns (labels, c1, c2)."""
    cost = refine_cost(disp, stable, dmax, lo, hi)
    agg = aggregate_twopass(forest["parent"], forest["wgt"], forest["order"], sigma,
                            np.nan_to_num(cost, nan=0.0))
    agg[np.isnan(cost)] = np.inf
    return wta(agg, lo, hi)


def stereo_level(left, right, dmax, level, pix_lo=None, pix_hi=None, beta=(19, 20),
                 sigma=0.1, prm=COST_PARAMS, sample_d=(), want_forest=True, rank=None):
    """One layer: forest, restricted cost, two-pass aggregation, WTA.
    rank: None (edges by colour weight) or one random number per grid edge
    [2N] (the random spanning tree RT of Section 4.1: edges by (rank, id))."""
    left = _c(left, np.float64); right = _c(right, np.float64)
    H, W = left.shape[:2]
    N = H * W
    disp = np.zeros(N, np.int32); c1 = np.zeros(N); c2 = np.zeros(N)
    outs = {}
    if want_forest:
        for k in ("parent", "depth", "order", "tree_lo", "tree_hi"):
            outs[k] = np.zeros(N, np.int32)
        outs["level_ptr"] = np.zeros(N + 1, np.int32)
    if pix_lo is not None:
        pix_lo = _c(pix_lo, np.int32).ravel(); pix_hi = _c(pix_hi, np.int32).ravel()
    sd = np.array(sample_d, np.int32)
    sa = np.zeros((len(sd), N), np.float64)
    pr = _prm(prm)
    g = outs.get
    nl = lib().or_stereo_level(_p(left), _p(right), H, W, dmax, level, _p(pix_lo), _p(pix_hi),
                               int(beta[0]), int(beta[1]), float(sigma), _p(pr),
                               _p(disp), _p(c1), _p(c2), _p(g("parent")), _p(g("depth")),
                               _p(g("order")), _p(g("level_ptr")), _p(g("tree_lo")),
                               _p(g("tree_hi")), len(sd), _p(sd if len(sd) else None),
                               _p(sa if len(sd) else None),
                               _p(None if rank is None else _c(rank, np.int64).ravel()))
    res = dict(disp=disp.reshape(H, W), c1=c1, c2=c2, n_levels=nl, sample_agg=sa)
    if want_forest:
        outs["level_ptr"] = outs["level_ptr"][:nl + 1].copy()
        res.update(outs)
    return res


def hdp_stereo(left_u8, right_u8, dmax, S=2, L=3, window=4, beta=(19, 20), sigma=0.1,
               prm=COST_PARAMS, want_forest=False, ranks=None):
    """Top-down HDP loop (Section 3): layer L over [0, d_L], then for l = L-1..0
    interval prediction, disparity forest, restricted cost, aggregation, WTA.
    ranks: None, or per layer l the random edge ranks [2 N_l] of HDP+RT.
    Returns a list of per-layer result dicts, index l."""
    H, W = left_u8.shape[:2]
    Hs, Ws, ds = level_dims(H, W, dmax, S, L)
    lp = pyramid(left_u8, S, L)
    rp = pyramid(right_u8, S, L)
    res = [None] * (L + 1)
    rk = (lambda l: None) if ranks is None else (lambda l: ranks[l])
    res[L] = stereo_level(lp[L], rp[L], ds[L], L, sigma=sigma, prm=prm, want_forest=want_forest,
                          rank=rk(L))
    res[L]["pix_lo"] = None; res[L]["pix_hi"] = None
    for l in range(L - 1, -1, -1):
        lo, hi = predict_range(res[l + 1]["disp"], Hs[l], Ws[l], S, window, ds[l])
        r = stereo_level(lp[l], rp[l], ds[l], l, lo, hi, beta=beta, sigma=sigma, prm=prm,
                         want_forest=want_forest, rank=rk(l))
        r["pix_lo"] = lo; r["pix_hi"] = hi
        res[l] = r
    return res


# --- gradients ---------------------------------------------------------------

def aggregate_grad_dense(H, W, in_tree, edge_w, sigma, cost, g):
    cost = _c(cost, np.float64); g = _c(g, np.float64)
    N, Dn = cost.shape
    dC = np.zeros_like(cost); dw = np.zeros(2 * N); ds = np.zeros(1)
    lib().or_aggregate_grad_dense(H, W, _p(_c(in_tree, np.uint8)),
                                  _p(_c(np.nan_to_num(edge_w, nan=0.0), np.float64)),
                                  float(sigma), Dn, _p(cost), _p(g), _p(dC), _p(dw), _p(ds))
    return dC, dw, float(ds[0])


def aggregate_backward_twopass(parent, wgt, order, sigma, cost, g):
    cost = _c(cost, np.float64); g = _c(g, np.float64)
    N, Dn = cost.shape
    dC = np.zeros_like(cost); dw = np.zeros(N); ds = np.zeros(1)
    lib().or_aggregate_backward_twopass(N, _p(_c(parent, np.int32)), _p(_c(wgt, np.float64)),
                                        _p(_c(order, np.int32)), float(sigma), Dn, _p(cost),
                                        _p(g), _p(dC), _p(dw), _p(ds))
    return dC, dw, float(ds[0])
