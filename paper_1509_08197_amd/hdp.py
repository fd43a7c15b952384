"""Thin Python binding of ``libhdp.so`` (argument marshalling only).

Every step runs in the HIP kernels behind the C ABI declared in
``include/hdp.h``; torch is used for device memory and streams.  There is no
CPU fallback: if the library is missing or no HIP device is present the calls
raise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdp.so")

MAX_PAIRS = 64
MAX_LABELS = 256
MAX_PHASES = 40
INFO_WORDS = 16
INFO = dict(n_levels=0, n_phases=1, n_trees=2, width=3, mst_rounds=4, rank_rounds=5,
            bad_interval=6, error=7, live_edges=8, active_components=9, tour_runs=10,
            list_edges=11)

STATUS = {0: "ok", -1: "invalid argument", -2: "invalid shape or batch",
          -3: "workspace too small", -4: "disparity forest not exact (an interval broke the bound given)",
          -5: "HIP runtime error"}


class HdpError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({code})")
        self.code = code


class Shape(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("dmax", C.c_int32)]


class CostParams(C.Structure):
    _fields_ = [("a_c", C.c_float), ("tau_c", C.c_float), ("a_g", C.c_float),
                ("tau_g", C.c_float), ("border", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("S", C.c_int32), ("L", C.c_int32), ("window", C.c_int32),
                ("beta_num", C.c_int32), ("beta_den", C.c_int32), ("sigma", C.c_float),
                ("cost", CostParams)]


MAX_GMM = 16


class Gmm(C.Structure):
    _fields_ = [("K", C.c_int32), ("pi", C.c_double * MAX_GMM), ("mu", C.c_double * MAX_GMM),
                ("sd", C.c_double * MAX_GMM)]


def make_gmm(pi, mu, sd) -> Gmm:
    """Mixture model GMM_l of the label offsets of one layer (Section 2.2)."""
    K = len(pi)
    assert 1 <= K <= MAX_GMM and len(mu) == K and len(sd) == K
    g = Gmm()
    g.K = K
    for k in range(K):
        g.pi[k], g.mu[k], g.sd[k] = float(pi[k]), float(mu[k]), float(sd[k])
    return g


class ForestStruct(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in (
        "parent", "depth", "tree", "lo", "hi", "row", "wgt", "order", "level_ptr", "node",
        "prow", "lc", "heavy", "rw", "phase_ptr", "info", "rx", "rlh")]


_lib = None


def lib():
    """Load libhdp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1509_08197_amd/build.py")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    P, I32, I64, F, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    L.hdp_forest_bytes.argtypes = [I64]; L.hdp_forest_bytes.restype = SZ
    L.hdp_forest_bind.argtypes = [P, SZ, I64, C.POINTER(ForestStruct)]
    L.hdp_level_shapes.argtypes = [P, I32, I32, I32, P]
    L.hdp_pyramid.argtypes = [P, P, I32, I32, I32, P, P]
    L.hdp_pyramid_views.argtypes = [P, P, P, I32, I32, I32, P, P, P]
    L.hdp_build_tree_workspace_bytes.argtypes = [I64]; L.hdp_build_tree_workspace_bytes.restype = SZ
    L.hdp_build_tree.argtypes = [P, P, I32, I32, P, P, I32, I32, I32, I32,
                                 C.POINTER(ForestStruct), P, SZ, P]
    L.hdp_build_random_tree.argtypes = [P, P, I32, I32, P, P, P, I32, I32, I32, I32,
                                        C.POINTER(ForestStruct), P, SZ, P]
    L.hdp_build_random_tree.restype = I32
    L.hdp_forest_read_info.argtypes = [C.POINTER(ForestStruct), P, P, P]
    L.hdp_level_order.argtypes = [C.POINTER(ForestStruct), P, SZ, P]
    L.hdp_cost_volume.argtypes = [P, P, P, I32, C.POINTER(ForestStruct), I32,
                                  C.POINTER(CostParams), P, P]
    L.hdp_aggregate_workspace_bytes.argtypes = [I64, I32]
    L.hdp_aggregate_workspace_bytes.restype = SZ
    L.hdp_aggregate.argtypes = [C.POINTER(ForestStruct), I32, P, F, P, P, P, SZ, P]
    L.hdp_aggregate_backward.argtypes = [C.POINTER(ForestStruct), I32, P, P, P, P, F,
                                         P, P, P, P, SZ, P]
    L.hdp_wta.argtypes = [C.POINTER(ForestStruct), P, I32, I32, P, P, P]
    L.hdp_match_layer.argtypes = [P, P, P, I32, C.POINTER(ForestStruct), I32,
                                  C.POINTER(CostParams), F, P, P, P, SZ, P]
    L.hdp_match_layer_noalloc.argtypes = [P, P, P, I32, C.POINTER(ForestStruct), I32,
                                          C.POINTER(CostParams), F, P, P, P]
    L.hdp_match_layer_noalloc.restype = I32
    L.hdp_match_layer_noalloc_max_bytes.argtypes = []
    L.hdp_match_layer_noalloc_max_bytes.restype = SZ
    L.hdp_interval_table.argtypes = [P, P, I32, I32, C.POINTER(Gmm), P, I32, C.c_double, P, P,
                                     I32, P, P]
    L.hdp_interval_table.restype = I32
    L.hdp_predict_range_table.argtypes = [P, P, P, I32, I32, P, P, I32, P, P, P]
    L.hdp_predict_range_table.restype = I32
    L.hdp_mirror.argtypes = [P, P, I32, P, P]
    L.hdp_lr_check.argtypes = [P, P, I32, P, I32, I32, P, P]
    L.hdp_sample_prior.argtypes = [P, P, P, I32, I32, P, I32, P]
    L.hdp_refine_cost.argtypes = [P, P, C.POINTER(ForestStruct), I32, P, P]
    for name in ("hdp_mirror", "hdp_lr_check", "hdp_sample_prior", "hdp_refine_cost"):
        getattr(L, name).restype = I32
    L.hdp_forest_set_weights.argtypes = [C.POINTER(ForestStruct), P, P]
    L.hdp_forest_set_weights.restype = I32
    L.hdp_predict_range.argtypes = [P, P, P, I32, I32, I32, P, P, P]
    L.hdp_status_str.argtypes = [I32]; L.hdp_status_str.restype = C.c_char_p
    L.hdp_timer_arm.argtypes = [I32]; L.hdp_timer_arm.restype = I32
    L.hdp_set_schedule.argtypes = [I32, I32, I32]; L.hdp_set_schedule.restype = I32
    L.hdp_plan_create.argtypes = [P, I32, C.POINTER(Params), C.POINTER(C.c_void_p)]
    L.hdp_plan_run.argtypes = [P, P, P, P, P]
    L.hdp_plan_layer.argtypes = [P, I32, C.POINTER(C.POINTER(ForestStruct)),
                                 C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(I32)]
    L.hdp_plan_inputs.argtypes = [P, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]
    L.hdp_plan_destroy.argtypes = [P]
    for name in ("hdp_plan_create", "hdp_plan_run", "hdp_plan_layer", "hdp_plan_inputs",
                 "hdp_plan_destroy"):
        getattr(L, name).restype = I32
    L.hdp_timer_read.argtypes = [P, P]; L.hdp_timer_read.restype = I32
    for name in ("hdp_forest_bind", "hdp_level_shapes", "hdp_pyramid", "hdp_build_tree",
                 "hdp_forest_read_info", "hdp_cost_volume", "hdp_aggregate",
                 "hdp_aggregate_backward", "hdp_wta", "hdp_predict_range"):
        getattr(L, name).restype = I32


def _check(fn, code):
    if code != 0:
        raise HdpError(fn, code)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _shapes(shapes: Sequence[Tuple[int, int, int]]):
    arr = (Shape * len(shapes))()
    for i, (H, W, d) in enumerate(shapes):
        arr[i].H, arr[i].W, arr[i].dmax = int(H), int(W), int(d)
    return arr


def n_pixels(shapes) -> int:
    return int(sum(int(H) * int(W) for H, W, _ in shapes))


def level_shapes(shapes, S: int, L: int) -> List[List[Tuple[int, int, int]]]:
    """Per level l = 0..L, the list of (H, W, dmax) of every pair (Section 2.1)."""
    n = len(shapes)
    out = (Shape * (n * (L + 1)))()
    _check("hdp_level_shapes", lib().hdp_level_shapes(_shapes(shapes), n, S, L, out))
    return [[(out[l * n + i].H, out[l * n + i].W, out[l * n + i].dmax) for i in range(n)]
            for l in range(L + 1)]


def _empty(nbytes, device):
    # 256-byte aligned device buffer (torch's allocator aligns to 512 B)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# --- pyramid ---------------------------------------------------------------------

def pyramid(rgb: torch.Tensor, shapes, S: int = 2, L: int = 3) -> List[torch.Tensor]:
    """rgb: uint8 [n0, 3] on the GPU (pairs concatenated).  Returns per level a
    float32 [n_l, 4] view (R, G, B, gx)."""
    assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.is_contiguous()
    lv = level_shapes(shapes, S, L)
    ns = [n_pixels(s) for s in lv]
    out = torch.empty((sum(ns), 4), dtype=torch.float32, device=rgb.device)
    _check("hdp_pyramid", lib().hdp_pyramid(_ptr(rgb), _shapes(shapes), len(shapes), S, L,
                                            _ptr(out), _stream()))
    views, off = [], 0
    for n in ns:
        views.append(out[off:off + n]); off += n
    return views


def pyramid_views(left_rgb: torch.Tensor, right_rgb: torch.Tensor, shapes, S: int = 2,
                  L: int = 3):
    """Pyramids of both views in the same launches; returns (left levels, right levels)."""
    for t in (left_rgb, right_rgb):
        assert t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous()
    lv = level_shapes(shapes, S, L)
    ns = [n_pixels(s) for s in lv]
    outs = [torch.empty((sum(ns), 4), dtype=torch.float32, device=left_rgb.device)
            for _ in range(2)]
    _check("hdp_pyramid_views", lib().hdp_pyramid_views(
        _ptr(left_rgb), _ptr(right_rgb), _shapes(shapes), len(shapes), S, L, _ptr(outs[0]),
        _ptr(outs[1]), _stream()))
    res = []
    for out in outs:
        views, off = [], 0
        for n in ns:
            views.append(out[off:off + n]); off += n
        res.append(views)
    return res[0], res[1]


# --- forest ----------------------------------------------------------------------

@dataclass
class Forest:
    buf: torch.Tensor
    st: ForestStruct
    n: int
    width: int
    shapes: list
    level: int
    info: Optional[List[int]] = None
    phase_ptr: Optional[List[int]] = None

    def _view(self, name, count, dtype):
        base = self.buf.data_ptr()
        off = getattr(self.st, name) - base
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.buf[off:off + count * esz].view(dtype)

    def array(self, name):
        n = self.n
        if name in ("parent", "depth", "tree", "lo", "hi", "row", "order", "node", "prow"):
            return self._view(name, n, torch.int32)
        if name in ("wgt", "rw"):
            return self._view(name, n, torch.float32)
        if name == "heavy":
            return self._view(name, n, torch.uint8)
        if name == "lc":
            return self._view(name, 2 * n, torch.int32).view(2, n)
        if name == "level_ptr":
            return self._view(name, n + 1, torch.int32)
        if name == "phase_ptr":
            return self._view(name, MAX_PHASES + 1, torch.int32)
        if name == "info":
            return self._view(name, INFO_WORDS, torch.int32)
        raise KeyError(name)

    def read_info(self):
        """Host copy of the scalars and the phase table (synchronises)."""
        info = (C.c_int32 * INFO_WORDS)()
        pp = (C.c_int32 * (MAX_PHASES + 1))()
        code = lib().hdp_forest_read_info(C.byref(self.st), info, pp, _stream())
        self.info = list(info)
        _check("hdp_forest_read_info", code)
        npz = self.info[INFO["n_phases"]]
        self.phase_ptr = list(pp)[:npz + 1]
        return self.info


def alloc_forest(n: int, device) -> Tuple[torch.Tensor, ForestStruct]:
    nbytes = lib().hdp_forest_bytes(n)
    buf = _empty(nbytes, device)
    st = ForestStruct()
    _check("hdp_forest_bind", lib().hdp_forest_bind(_ptr(buf), nbytes, n, C.byref(st)))
    return buf, st


class Workspace:
    """Grow-only scratch buffer reused across calls (no allocation when large enough)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = _empty(nbytes, device)
        return self.buf


_ws_tree = Workspace()
_ws_agg = Workspace()


def build_tree(img: torch.Tensor, shapes, level: int, pix_lo=None, pix_hi=None,
               max_width: int = 0, beta=(19, 20), width: Optional[int] = None,
               read_info: bool = False, forest: Optional[Forest] = None, ws=None,
               level_order: bool = True, rank: Optional[torch.Tensor] = None) -> Forest:
    """Minimum spanning tree (pix_lo None) or disparity forest of one layer.
    rank: None, or int32 [2n] random edge ranks: the random spanning tree RT
    (and its disparity forest) instead of the MST.
    level_order: also fill the canonical (depth, id) order and level_ptr."""
    n = n_pixels(shapes)
    assert img.shape == (n, 4) and img.dtype == torch.float32 and img.is_contiguous()
    if width is None:
        dfull = max(d for _, _, d in shapes) + 1
        if pix_lo is None:
            width = dfull
        elif beta[0] * max_width <= beta[1] * (max_width - 1):
            # outside the exact regime the sequential process runs and merges
            # can widen a tree's interval up to the full range
            width = dfull
        else:
            width = max_width
    dev = img.device
    if forest is None:
        buf, st = alloc_forest(n, dev)
        forest = Forest(buf=buf, st=st, n=n, width=width, shapes=list(shapes), level=level)
    else:
        forest.width = width
        forest.shapes = list(shapes)
        forest.level = level
    wsb = lib().hdp_build_tree_workspace_bytes(n)
    w = (ws or _ws_tree).get(wsb, dev)
    if rank is None:
        _check("hdp_build_tree", lib().hdp_build_tree(
            _ptr(img), _shapes(shapes), len(shapes), level, _ptr(pix_lo), _ptr(pix_hi),
            int(max_width), int(beta[0]), int(beta[1]), int(width), C.byref(forest.st), _ptr(w),
            wsb, _stream()))
    else:
        assert rank.shape == (2 * n,) and rank.dtype == torch.int32 and rank.is_contiguous()
        _check("hdp_build_random_tree", lib().hdp_build_random_tree(
            _ptr(img), _shapes(shapes), len(shapes), level, _ptr(rank), _ptr(pix_lo),
            _ptr(pix_hi), int(max_width), int(beta[0]), int(beta[1]), int(width),
            C.byref(forest.st), _ptr(w), wsb, _stream()))
    if level_order:
        _check("hdp_level_order",
               lib().hdp_level_order(C.byref(forest.st), _ptr(w), wsb, _stream()))
    if read_info:
        forest.read_info()
    return forest


def set_weights(forest: Forest, wgt: torch.Tensor):
    """Load per-pixel edge weights (edge to the parent) into the forest."""
    assert wgt.shape == (forest.n,) and wgt.dtype == torch.float32 and wgt.is_contiguous()
    _check("hdp_forest_set_weights",
           lib().hdp_forest_set_weights(C.byref(forest.st), _ptr(wgt), _stream()))


# --- cost, aggregation, WTA ---------------------------------------------------------

def cost_params(a_c=0.89, tau_c=7.0, a_g=0.11, tau_g=2.0, border=0) -> CostParams:
    """border 0: a label past the left image border costs both truncations;
    1: it is compared with the row's first pixel."""
    return CostParams(a_c, tau_c, a_g, tau_g, border)


def cost_volume(left: torch.Tensor, right: torch.Tensor, shapes, forest: Optional[Forest] = None,
                width: Optional[int] = None, params: Optional[CostParams] = None,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = n_pixels(shapes)
    if width is None:
        width = forest.width if forest is not None else max(d for _, _, d in shapes) + 1
    if out is None:
        out = torch.empty((n, width), dtype=torch.float32, device=left.device)
    p = params or cost_params()
    _check("hdp_cost_volume", lib().hdp_cost_volume(
        _ptr(left), _ptr(right), _shapes(shapes), len(shapes),
        C.byref(forest.st) if forest is not None else None, int(width), C.byref(p), _ptr(out),
        _stream()))
    return out


def aggregate(forest: Forest, cost: torch.Tensor, sigma: float = 0.1, keep_up: bool = False,
              out: Optional[torch.Tensor] = None, up: Optional[torch.Tensor] = None, ws=None):
    """agg(v,x) = sum_u exp(-W(v,u)/sigma) cost(u,x) over the forest (eq. C).
    Returns agg, or (agg, U) with keep_up."""
    n, width = forest.n, forest.width
    assert cost.shape == (n, width) and cost.dtype == torch.float32 and cost.is_contiguous()
    if out is None:
        out = torch.empty_like(cost)
    if keep_up and up is None:
        up = torch.empty_like(cost)
    wsb = lib().hdp_aggregate_workspace_bytes(n, width)
    w = (ws or _ws_agg).get(wsb, cost.device)
    _check("hdp_aggregate", lib().hdp_aggregate(
        C.byref(forest.st), width, _ptr(cost), float(sigma), _ptr(out), _ptr(up),
        _ptr(w), wsb, _stream()))
    return (out, up) if keep_up else out


def aggregate_backward(forest: Forest, cost, agg, grad_agg, sigma=0.1, up=None,
                       want_w=True, want_sigma=True, ws=None):
    """Returns (grad_cost, grad_w per pixel or None, grad_sigma tensor or None)."""
    n, width = forest.n, forest.width
    gc = torch.empty_like(cost)
    gw = torch.zeros(n, dtype=torch.float32, device=cost.device) if want_w else None
    gs = torch.zeros(1, dtype=torch.float32, device=cost.device) if want_sigma else None
    wsb = lib().hdp_aggregate_workspace_bytes(n, width)
    w = (ws or _ws_agg).get(wsb, cost.device)
    _check("hdp_aggregate_backward", lib().hdp_aggregate_backward(
        C.byref(forest.st), width, _ptr(cost), _ptr(agg), _ptr(up),
        _ptr(grad_agg.contiguous()), float(sigma), _ptr(gc), _ptr(gw), _ptr(gs), _ptr(w), wsb,
        _stream()))
    return gc, gw, gs


def wta(agg: torch.Tensor, shapes, forest: Optional[Forest] = None,
        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = n_pixels(shapes)
    width = agg.shape[1]
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=agg.device)
    _check("hdp_wta", lib().hdp_wta(C.byref(forest.st) if forest is not None else None,
                                    _shapes(shapes), len(shapes), int(width), _ptr(agg), _ptr(out),
                                    _stream()))
    return out


def match_layer(left: torch.Tensor, right: torch.Tensor, shapes, forest: Forest,
                sigma: float = 0.1, params: Optional[CostParams] = None, agg=None, disp=None,
                ws=None):
    """Cost, aggregation and WTA of one layer in one call (fused passes for
    rows of at most 64 labels, or up to 256 in multiples of four).  Returns
    (agg, disp)."""
    n, width = forest.n, forest.width
    if agg is None:
        agg = torch.empty((n, width), dtype=torch.float32, device=left.device)
    if disp is None:
        disp = torch.empty(n, dtype=torch.int32, device=left.device)
    p = params or cost_params()
    wsb = lib().hdp_aggregate_workspace_bytes(n, width)
    w = (ws or _ws_agg).get(wsb, left.device)
    _check("hdp_match_layer", lib().hdp_match_layer(
        _ptr(left), _ptr(right), _shapes(shapes), len(shapes), C.byref(forest.st), int(width),
        C.byref(p), float(sigma), _ptr(agg), _ptr(disp), _ptr(w), wsb, _stream()))
    return agg, disp


def match_layer_noalloc(left: torch.Tensor, right: torch.Tensor, shapes, forest: Forest,
                        sigma: float = 0.1, params: Optional[CostParams] = None, agg=None,
                        disp=None):
    """match_layer with the library's fixed scratch array instead of a
    workspace (the call allocates nothing on the device).  Returns (agg, disp)."""
    n, width = forest.n, forest.width
    if agg is None:
        agg = torch.empty((n, width), dtype=torch.float32, device=left.device)
    if disp is None:
        disp = torch.empty(n, dtype=torch.int32, device=left.device)
    p = params or cost_params()
    _check("hdp_match_layer_noalloc", lib().hdp_match_layer_noalloc(
        _ptr(left), _ptr(right), _shapes(shapes), len(shapes), C.byref(forest.st), int(width),
        C.byref(p), float(sigma), _ptr(agg), _ptr(disp), _stream()))
    return agg, disp


def noalloc_max_bytes() -> int:
    """Size of the fixed scratch array behind match_layer_noalloc."""
    return int(lib().hdp_match_layer_noalloc_max_bytes())


def predict_range(disp_upper: torch.Tensor, upper_shapes, lower_shapes, S: int = 2,
                  window: int = 4, out=None):
    n = n_pixels(lower_shapes)
    if out is None:
        lo = torch.empty(n, dtype=torch.int32, device=disp_upper.device)
        hi = torch.empty(n, dtype=torch.int32, device=disp_upper.device)
    else:
        lo, hi = out
    _check("hdp_predict_range", lib().hdp_predict_range(
        _ptr(disp_upper), _shapes(upper_shapes), _shapes(lower_shapes), len(lower_shapes), S,
        window, _ptr(lo), _ptr(hi), _stream()))
    return lo, hi


def interval_table(upper_shapes, lower_shapes, S: int, gmm: Gmm, prior: torch.Tensor,
                   delta: float):
    """Bayesian interval table of one layer (Section 2.2 eq. dpm, Section 3.1
    eq. crtr).  prior: float64 [n_pairs, stride] on the GPU (P(D_l = j) per
    pair).  Returns (lo_tab, hi_tab, max_width) with the tables int32
    [n_pairs, d_up + 1] and max_width a 1-element device tensor."""
    assert prior.dtype == torch.float64 and prior.is_cuda and prior.is_contiguous()
    n = len(lower_shapes)
    assert prior.shape[0] == n
    tab_stride = max(d for _, _, d in upper_shapes) + 1
    lo = torch.empty((n, tab_stride), dtype=torch.int32, device=prior.device)
    hi = torch.empty_like(lo)
    mw = torch.empty(1, dtype=torch.int32, device=prior.device)
    _check("hdp_interval_table", lib().hdp_interval_table(
        _shapes(upper_shapes), _shapes(lower_shapes), n, S, C.byref(gmm), _ptr(prior),
        int(prior.shape[1]), float(delta), _ptr(lo), _ptr(hi), tab_stride, _ptr(mw), _stream()))
    return lo, hi, mw


def predict_range_table(disp_upper: torch.Tensor, upper_shapes, lower_shapes, S: int,
                        lo_tab: torch.Tensor, hi_tab: torch.Tensor, out=None):
    n = n_pixels(lower_shapes)
    if out is None:
        lo = torch.empty(n, dtype=torch.int32, device=disp_upper.device)
        hi = torch.empty(n, dtype=torch.int32, device=disp_upper.device)
    else:
        lo, hi = out
    _check("hdp_predict_range_table", lib().hdp_predict_range_table(
        _ptr(disp_upper), _shapes(upper_shapes), _shapes(lower_shapes), len(lower_shapes), S,
        _ptr(lo_tab), _ptr(hi_tab), int(lo_tab.shape[1]), _ptr(lo), _ptr(hi), _stream()))
    return lo, hi


# --- left-right check, sampled prior, refinement (Sections 3.1, 3.3) ------------------

def mirror(rgb: torch.Tensor, shapes) -> torch.Tensor:
    """Every pair's image flipped left to right (uint8 [n, 3])."""
    assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.is_contiguous()
    out = torch.empty_like(rgb)
    _check("hdp_mirror", lib().hdp_mirror(_ptr(rgb), _shapes(shapes), len(shapes), _ptr(out),
                                          _stream()))
    return out


def right_view(left_rgb, right_rgb, shapes, **kw):
    """The method run on the mirrored pair with the right image as reference:
    the right view's labels, in mirrored coordinates (see lr_check)."""
    return hdp_stereo(mirror(right_rgb, shapes), mirror(left_rgb, shapes), shapes, **kw)


def lr_check(disp_left: torch.Tensor, disp_right: torch.Tensor, shapes, tol: int = 0,
             right_mirrored: bool = True) -> torch.Tensor:
    """Stable pixels (uint8 0/1) of the left view (left-right consistency)."""
    out = torch.empty(disp_left.shape, dtype=torch.uint8, device=disp_left.device)
    _check("hdp_lr_check", lib().hdp_lr_check(_ptr(disp_left), _ptr(disp_right),
                                              1 if right_mirrored else 0, _shapes(shapes),
                                              len(shapes), int(tol), _ptr(out), _stream()))
    return out


def sample_prior(disp: torch.Tensor, stable: torch.Tensor, shapes, square: int = 5,
                 stride: Optional[int] = None) -> torch.Tensor:
    """P(D_l) per pair: counts of the labels of the stable block centres
    (float64 [n_pairs, stride], Section 3.1)."""
    stride = stride or max(d for _, _, d in shapes) + 1
    out = torch.empty((len(shapes), stride), dtype=torch.float64, device=disp.device)
    _check("hdp_sample_prior", lib().hdp_sample_prior(
        _ptr(disp), _ptr(stable), _shapes(shapes), len(shapes), int(square), _ptr(out), stride,
        _stream()))
    return out


def refine(forest: Forest, disp: torch.Tensor, stable: torch.Tensor, sigma: float = 0.1,
           ws=None):
    """Tree-based refinement of one layer's labels over its forest (Section 3.3):
    refinement cost, aggregation, winner-takes-all.  Returns (agg, labels)."""
    cost = torch.empty((forest.n, forest.width), dtype=torch.float32, device=disp.device)
    _check("hdp_refine_cost", lib().hdp_refine_cost(_ptr(disp), _ptr(stable), C.byref(forest.st),
                                                    int(forest.width), _ptr(cost), _stream()))
    agg = aggregate(forest, cost, sigma, ws=ws)
    return agg, wta(agg, forest.shapes, forest)


# --- diagnostics -----------------------------------------------------------------------

TIMER = dict(up_pass=0, down_pass=1, cost=2)


def set_schedule(width: int, labels_per_thread: int, rows_per_group: int = 8):
    """Tile schedule of the aggregation passes for rows of `width` labels
    (labels_per_thread = 0 restores the built-in choice)."""
    _check("hdp_set_schedule", lib().hdp_set_schedule(int(width), int(labels_per_thread),
                                                      int(rows_per_group)))


def timer_arm(kernel_class: Optional[str]):
    """Record HIP events around every launch of one kernel class (None: off)."""
    _check("hdp_timer_arm", lib().hdp_timer_arm(-1 if kernel_class is None else TIMER[kernel_class]))


def timer_read() -> Tuple[float, int]:
    """(summed kernel milliseconds, launches) of the armed class; synchronises."""
    ms = C.c_float(); n = C.c_int32()
    _check("hdp_timer_read", lib().hdp_timer_read(C.byref(ms), C.byref(n)))
    return float(ms.value), int(n.value)


# --- the method ----------------------------------------------------------------------

@dataclass
class LevelResult:
    level: int
    shapes: list
    forest: Forest
    disp: torch.Tensor
    pix_lo: Optional[torch.Tensor] = None
    pix_hi: Optional[torch.Tensor] = None
    cost: Optional[torch.Tensor] = None
    agg: Optional[torch.Tensor] = None


def stereo_level(left_img, right_img, shapes, level, pix_lo=None, pix_hi=None, max_width=0,
                 beta=(19, 20), sigma=0.1, params=None, keep=False, ws=None,
                 rank=None) -> LevelResult:
    """One layer (Section 3): forest, restricted cost, aggregation, WTA.
    keep: run the three steps apart and also return the cost and aggregated
    volumes (and fill the forest's level order); otherwise one fused call.
    rank: random edge ranks of the layer (random spanning tree RT) or None."""
    ws = ws or {}
    f = build_tree(left_img, shapes, level, pix_lo, pix_hi, max_width=max_width, beta=beta,
                   read_info=False, ws=ws.get("tree"), level_order=keep, rank=rank)
    if not keep:
        agg, disp = match_layer(left_img, right_img, shapes, f, sigma, params, ws=ws.get("agg"))
        return LevelResult(level=level, shapes=list(shapes), forest=f, disp=disp, pix_lo=pix_lo,
                           pix_hi=pix_hi, cost=None, agg=None)
    cost = cost_volume(left_img, right_img, shapes, f, params=params)
    agg = aggregate(f, cost, sigma, ws=ws.get("agg"))
    disp = wta(agg, shapes, f)
    return LevelResult(level=level, shapes=list(shapes), forest=f, disp=disp, pix_lo=pix_lo,
                       pix_hi=pix_hi, cost=cost, agg=agg)


def hdp_stereo(left_rgb: torch.Tensor, right_rgb: torch.Tensor, shapes, S=2, L=3, window=4,
               beta=(19, 20), sigma=0.1, params=None, keep=False, ws=None,
               ranks=None, gmm=None, priors=None, delta0=0.004,
               gmm_max_width=None) -> List[LevelResult]:
    """Top-down HDP (Section 3): layer L over [0, d_L] with the MST, then for
    l = L-1..0 interval prediction -> disparity forest -> cost -> aggregation
    -> WTA.  left_rgb/right_rgb: uint8 [n0, 3].  ranks: None (MST), or per
    layer the random edge ranks of HDP+RT (see draw_edge_ranks).

    Interval prediction: the window [S i - window, S i + S - 1 + window] by
    default; with gmm (per layer l < L a Gmm, see make_gmm) and priors (per
    layer l < L a float64 [n_pairs, stride] device tensor of P(D_l)), the
    Bayesian table with delta_l = delta0 * S^l.  gmm_max_width: a bound on the
    table's widths (then nothing synchronises); None reads the widest interval
    back from the device.  Returns results indexed by layer."""
    lv = level_shapes(shapes, S, L)
    lp, rp = pyramid_views(left_rgb, right_rgb, shapes, S, L)
    rk = (lambda l: None) if ranks is None else (lambda l: ranks[l])
    res: List[Optional[LevelResult]] = [None] * (L + 1)
    res[L] = stereo_level(lp[L], rp[L], lv[L], L, sigma=sigma, params=params, keep=keep, ws=ws,
                          rank=rk(L))
    for l in range(L - 1, -1, -1):
        dl = max(d for _, _, d in lv[l])
        if gmm is None:
            lo, hi = predict_range(res[l + 1].disp, lv[l + 1], lv[l], S, window)
            mw = min(S + 2 * window, dl + 1)
        else:
            lo_t, hi_t, mwt = interval_table(lv[l + 1], lv[l], S, gmm[l], priors[l],
                                             delta0 * S ** l)
            lo, hi = predict_range_table(res[l + 1].disp, lv[l + 1], lv[l], S, lo_t, hi_t)
            mw = int(mwt.item()) if gmm_max_width is None else min(int(gmm_max_width), dl + 1)
        res[l] = stereo_level(lp[l], rp[l], lv[l], l, lo, hi, max_width=mw, beta=beta,
                              sigma=sigma, params=params, keep=keep, ws=ws, rank=rk(l))
    return res


def draw_edge_ranks(shapes, S: int = 2, L: int = 3, generator=None, device="cuda"):
    """One random int32 rank in [0, 2^31) per grid edge (2 per pixel) of every
    layer: the random shuffle of the random spanning tree RT (Section 4.1).
    Returns a list indexed by layer."""
    out = []
    for lvl in level_shapes(shapes, S, L):
        n = n_pixels(lvl)
        out.append(torch.randint(0, 2 ** 31 - 1, (2 * n,), dtype=torch.int32, device=device,
                                 generator=generator))
    return out


def full_range(left_rgb, right_rgb, shapes, sigma=0.1, params=None, keep=False,
               ws=None, rank=None) -> LevelResult:
    """Full-range MST (or, with rank, RT) aggregation + WTA at the input
    resolution (the baseline the method speeds up)."""
    lp, rp = pyramid_views(left_rgb, right_rgb, shapes, 2, 0)
    return stereo_level(lp[0], rp[0], shapes, 0, sigma=sigma, params=params, keep=keep, ws=ws,
                        rank=rank)


class CapturedStep:
    """A whole step captured once into a HIP graph and replayed.

    ``fn(ws)`` must enqueue only library calls on the current stream (no host
    synchronisation).  The step owns its workspaces, so no other call can
    reallocate memory the graph refers to.  Inputs are read from the tensors
    captured by ``fn``; overwrite them in place between replays."""

    def __init__(self, fn, warmup: int = 1):
        self.ws = {"tree": Workspace(), "agg": Workspace()}
        self.stream = torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                fn(self.ws)
        torch.cuda.current_stream().wait_stream(self.stream)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.out = fn(self.ws)

    def replay(self):
        self.graph.replay()
        return self.out


_hip = None


def _hip_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy on the current stream (HIP runtime)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    if _hip.hipMemcpyAsync(C.c_void_p(dst), C.c_void_p(src), nbytes, 3, _stream()) != 0:
        raise HdpError("hipMemcpyAsync", -5)


class Plan:
    """Native batch plan (C ABI hdp_plan_*): the whole top-down loop for a fixed
    batch, buffers allocated once, one HIP graph launch per run."""

    def __init__(self, shapes, S=2, L=3, window=4, beta=(19, 20), sigma=0.1, params=None):
        self.shapes = list(shapes)
        self.n0 = n_pixels(shapes)
        p = Params(S, L, window, beta[0], beta[1], sigma, params or cost_params())
        h = C.c_void_p()
        _check("hdp_plan_create", lib().hdp_plan_create(_shapes(shapes), len(shapes), C.byref(p),
                                                        C.byref(h)))
        self.h = h
        self.L = L

    def run(self, left_rgb=None, right_rgb=None, disp: Optional[torch.Tensor] = None):
        _check("hdp_plan_run", lib().hdp_plan_run(self.h, _ptr(left_rgb), _ptr(right_rgb),
                                                  _ptr(disp), _stream()))
        return disp

    def layer_disp(self, level: int) -> torch.Tensor:
        """Copy of the labels of one layer (after a run)."""
        f = C.POINTER(ForestStruct)()
        d = C.c_void_p()
        _check("hdp_plan_layer", lib().hdp_plan_layer(self.h, level, C.byref(f), C.byref(d), None,
                                                      None))
        n = f.contents.n
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        _hip_d2d(out.data_ptr(), d.value, 4 * n)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().hdp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
