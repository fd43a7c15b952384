"""Seeded synthetic stereo pairs shaped like the paper's benchmark images.

This module only draws inputs: textures, ground-truth disparity maps and the
right view obtained by warping the left one.  It contains none of the stereo
method's arithmetic (no pyramid, cost, tree or aggregation), so both the CPU
oracle and the GPU path can be fed from it.

The paper evaluates on Middlebury 2006 full size (width 1240-1396, height
1110), on KITTI frames (1242x375) and on its own 640x480 web-camera pairs
(Section 4.1).  None of those datasets is available here; the scenes below are
synthetic stand-ins with the same image shapes and disparity ranges.

Recipe (all randomness from ``numpy.random.default_rng(seed)``):

* texture: per channel, multi-octave value noise with lattice spacings
  64/32/16/8/4 px, smoothstep-weighted bilinear interpolation, amplitude halved
  per octave, mapped linearly to [16, 240];
* ground truth: scene-specific (rectangles over a background, slanted planar
  Voronoi cells, or a road plane with upright boxes);
* right view: forward splat of the left view by the rounded ground-truth
  disparity (x_r = x - d); where several left pixels land on one right pixel
  the larger disparity (closer surface) wins; holes are filled with a fresh
  texture drawn from a different seed;
* sensor noise: independent Gaussian noise on both views, rounded and clipped
  to uint8.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SPACINGS = (64, 32, 16, 8, 4)


@dataclass
class StereoPair:
    left: np.ndarray    # (H, W, 3) uint8
    right: np.ndarray   # (H, W, 3) uint8
    gt: np.ndarray      # (H, W) float64 ground-truth disparity of the left view
    dmax: int           # labels are 0..dmax

    @property
    def shape(self):
        return self.left.shape[0], self.left.shape[1]


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise(rng: np.random.Generator, H: int, W: int, spacings=SPACINGS) -> np.ndarray:
    """One channel of multi-octave value noise in [0, 1]."""
    out = np.zeros((H, W), dtype=np.float64)
    total = 0.0
    amp = 1.0
    for s in spacings:
        gh, gw = H // s + 2, W // s + 2
        lat = rng.random((gh, gw))
        y = np.arange(H, dtype=np.float64) / s
        x = np.arange(W, dtype=np.float64) / s
        y0 = np.floor(y).astype(np.int64)
        x0 = np.floor(x).astype(np.int64)
        fy = _smoothstep(y - y0)[:, None]
        fx = _smoothstep(x - x0)[None, :]
        v00 = lat[y0][:, x0]
        v01 = lat[y0][:, x0 + 1]
        v10 = lat[y0 + 1][:, x0]
        v11 = lat[y0 + 1][:, x0 + 1]
        top = v00 + (v01 - v00) * fx
        bot = v10 + (v11 - v10) * fx
        out += amp * (top + (bot - top) * fy)
        total += amp
        amp *= 0.5
    return out / total


def texture(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """(H, W, 3) float texture in [16, 240]."""
    return np.stack([16.0 + 224.0 * value_noise(rng, H, W) for _ in range(3)], axis=-1)


def warp_right(left_tex: np.ndarray, gt: np.ndarray, fill_seed: int) -> np.ndarray:
    """Forward-splat the left texture to the right view (x_r = x - round(d))."""
    H, W, _ = left_tex.shape
    d = np.rint(gt).astype(np.int64)
    ys, xs = np.mgrid[0:H, 0:W]
    xr = xs - d
    ok = xr >= 0
    # z-buffer: larger disparity wins.  Sort by disparity so later writes win.
    yy, xx, dd, xrr = ys[ok], xs[ok], d[ok], xr[ok]
    idx = np.argsort(dd, kind="stable")
    yy, xx, xrr = yy[idx], xx[idx], xrr[idx]
    right = texture(np.random.default_rng(fill_seed), H, W)
    filled = np.zeros((H, W), dtype=bool)
    right[yy, xrr] = left_tex[yy, xx]
    filled[yy, xrr] = True
    return right


def _finish(rng, left_tex, right_tex, gt, dmax, sigma_noise) -> StereoPair:
    H, W, _ = left_tex.shape
    nl = rng.normal(0.0, sigma_noise, size=(H, W, 3))
    nr = rng.normal(0.0, sigma_noise, size=(H, W, 3))
    left = np.clip(np.rint(left_tex + nl), 0, 255).astype(np.uint8)
    right = np.clip(np.rint(right_tex + nr), 0, 255).astype(np.uint8)
    return StereoPair(left=left, right=right, gt=gt, dmax=int(dmax))


def rectangles_scene(seed: int, H: int = 120, W: int = 160, dmax: int = 15,
                     sigma_noise: float = 2.0) -> StereoPair:
    """Fronto-parallel rectangles over a constant background disparity."""
    rng = np.random.default_rng(seed)
    bg = int(rng.integers(0, min(3, dmax) + 1))
    gt = np.full((H, W), float(bg))
    n = int(rng.integers(3, 7))
    for _ in range(n):
        rw = int(rng.integers(max(1, W // 8), max(2, W // 2) + 1))
        rh = int(rng.integers(max(1, H // 8), max(2, H // 2) + 1))
        x0 = int(rng.integers(0, W - rw + 1))
        y0 = int(rng.integers(0, H - rh + 1))
        dv = int(rng.integers(min(bg + 1, dmax), dmax + 1))
        gt[y0:y0 + rh, x0:x0 + rw] = dv
    tex = texture(rng, H, W)
    right = warp_right(tex, gt, fill_seed=seed + 7_000_003)
    return _finish(rng, tex, right, gt, dmax, sigma_noise)


def planes_scene(seed: int, H: int = 1104, W: int = 1344, dmax: int = 255,
                 sigma_noise: float = 2.0) -> StereoPair:
    """20-40 Voronoi cells, each a slanted plane d = a(x-cx) + b(y-cy) + c."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 41))
    cx = rng.uniform(0, W, n)
    cy = rng.uniform(0, H, n)
    a = rng.uniform(-0.3, 0.3, n)
    b = rng.uniform(-0.3, 0.3, n)
    c = rng.uniform(0, dmax, n)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int64)
    for k in range(n):
        d2 = (xs - cx[k]) ** 2 + (ys - cy[k]) ** 2
        m = d2 < best
        best[m] = d2[m]
        lab[m] = k
    gt = a[lab] * (xs - cx[lab]) + b[lab] * (ys - cy[lab]) + c[lab]
    gt = np.clip(gt, 0.0, float(dmax))
    tex = texture(rng, H, W)
    right = warp_right(tex, gt, fill_seed=seed + 7_000_003)
    return _finish(rng, tex, right, gt, dmax, sigma_noise)


def road_scene(seed: int, H: int = 375, W: int = 1242, dmax: int = 191,
               sigma_noise: float = 3.0) -> StereoPair:
    """Road-like ground plane d(y) = dmax*y/(H-1) plus 10-30 upright boxes."""
    rng = np.random.default_rng(seed)
    ys = np.arange(H, dtype=np.float64)
    ground = dmax * ys / max(H - 1, 1)
    gt = np.repeat(ground[:, None], W, axis=1)
    n = int(rng.integers(10, 31))
    boxes = []
    for _ in range(n):
        yb = int(rng.integers(H // 3, H))
        bh = int(rng.integers(max(2, H // 12), max(3, H // 3) + 1))
        bw = int(rng.integers(max(2, W // 40), max(3, W // 8) + 1))
        x0 = int(rng.integers(0, max(1, W - bw)))
        boxes.append((yb, bh, bw, x0))
    # farther boxes first so that closer ones overwrite them
    for yb, bh, bw, x0 in sorted(boxes, key=lambda t: t[0]):
        y0 = max(0, yb - bh)
        gt[y0:yb + 1, x0:x0 + bw] = ground[yb]
    tex = texture(rng, H, W)
    right = warp_right(tex, gt, fill_seed=seed + 7_000_003)
    return _finish(rng, tex, right, gt, dmax, sigma_noise)


# --- the five workloads ------------------------------------------------------

def config_seed(cfg: int, pair: int) -> int:
    return 1000 * cfg + pair


def workload(cfg: int, pair: int = 0) -> StereoPair:
    """Pair ``pair`` of workload ``cfg`` (1..5), seeded by 1000*cfg + pair."""
    seed = config_seed(cfg, pair)
    if cfg == 1:
        return rectangles_scene(seed, H=120, W=160, dmax=15, sigma_noise=2.0)
    if cfg == 2:
        return planes_scene(seed, H=1104, W=1344, dmax=255, sigma_noise=2.0)
    if cfg == 3:
        rng = np.random.default_rng(seed + 500)
        W = int(rng.integers(320, 1393))
        H = int(rng.integers(240, 1111))
        labels = int(rng.choice([64, 128, 192, 256]))
        return planes_scene(seed, H=H, W=W, dmax=labels - 1, sigma_noise=2.0)
    if cfg == 4:
        return planes_scene(seed, H=480, W=640, dmax=127, sigma_noise=2.0)
    if cfg == 5:
        return road_scene(seed, H=375, W=1242, dmax=191, sigma_noise=3.0)
    raise ValueError(f"unknown workload {cfg}")


# Per-workload pyramid/prediction parameters: (levels L, window w, beta num/den).
HDP_PARAMS = {
    2: dict(S=2, L=3, window=4, beta=(19, 20)),
    3: dict(S=2, L=3, window=4, beta=(19, 20)),
    5: dict(S=2, L=2, window=6, beta=(19, 20)),
}

N_PAIRS = {1: 1, 2: 1, 3: 32, 4: 8, 5: 64}


def small_scene(seed: int, H: int, W: int, dmax: int, sigma_noise: float = 2.0) -> StereoPair:
    """Slanted-plane scene at an arbitrary (small) size, for tests."""
    return planes_scene(seed, H=H, W=W, dmax=dmax, sigma_noise=sigma_noise)


def gmm_params(seed: int, L: int, K: int = 3, sd_range=(0.3, 0.7)):
    """Stand-ins for the trained mixture models GMM_l (Section 2.2) of the label
    offset o = D_{l+1} - floor(D_l / S), one per layer l < L: K components with
    weights from a flat Dirichlet draw, means uniform in [-0.5, 0.5] and
    standard deviations uniform in sd_range.  (The paper trains them by EM on
    Middlebury ground truth and does not print them.)  Returns a list of
    (pi, mu, sd) arrays."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(L):
        pi = rng.dirichlet(np.ones(K))
        mu = rng.uniform(-0.5, 0.5, K)
        sd = rng.uniform(sd_range[0], sd_range[1], K)
        out.append((pi, mu, sd))
    return out


def label_prior(gt: np.ndarray, S: int, level: int, dmax_l: int, square: int = 5) -> np.ndarray:
    """Stand-in for the sampled distribution P(D_l) of Section 3.1: the paper
    takes the disparities of the centres of 5x5 squares of layer l (computed
    and checked for left-right consistency); here the ground truth at those
    centres, in layer-l labels floor(d / S^l), counted per label 0..dmax_l."""
    f = S ** level
    Hl, Wl = -(-gt.shape[0] // f), -(-gt.shape[1] // f)
    ys = np.arange(square // 2, Hl, square)
    xs = np.arange(square // 2, Wl, square)
    d = gt[np.minimum(ys * f, gt.shape[0] - 1)][:, np.minimum(xs * f, gt.shape[1] - 1)]
    lab = np.clip(np.floor(d / f).astype(np.int64), 0, dmax_l)
    return np.bincount(lab.ravel(), minlength=dmax_l + 1).astype(np.float64)


def random_cost(seed: int, n_rows: int, width: int) -> np.ndarray:
    """Non-negative float32 cost rows (exactly representable values)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 1 << 16, size=(n_rows, width)).astype(np.float32) / np.float32(4096.0))


def _workload_args(args):
    return workload(*args)


def _gpu_initialised() -> bool:
    """True once this process has made a HIP call through torch (a fork after
    that point would hand the children the parent's device state)."""
    import sys
    torch = sys.modules.get("torch")
    return bool(torch is not None and torch.cuda.is_initialized())


_BATCHES = {}


def prefetch(cfgs, processes: int = 16) -> None:
    """Draw the pairs of the batched workloads ``cfgs`` now and keep them for
    ``workload_batch``.  Called before the process's first GPU call, it draws
    them in forked host processes; afterwards it draws them one by one here."""
    for cfg in cfgs:
        if cfg not in _BATCHES:
            _BATCHES[cfg] = _draw_batch(cfg, N_PAIRS[cfg], processes)


def _draw_batch(cfg: int, n: int, processes: int):
    if n == 1 or processes <= 1 or _gpu_initialised():
        return [workload(cfg, i) for i in range(n)]
    from multiprocessing import get_context
    with get_context("fork").Pool(min(processes, n)) as pool:
        return pool.map(_workload_args, [(cfg, i) for i in range(n)])


def workload_batch(cfg: int, n: int = None, processes: int = 16):
    """All pairs of a batched workload: the prefetched ones if ``prefetch`` drew
    them, otherwise drawn now (in forked host processes only while the process
    has not touched the GPU)."""
    n = N_PAIRS[cfg] if n is None else n
    if cfg in _BATCHES and len(_BATCHES[cfg]) >= n:
        return _BATCHES[cfg][:n]
    return _draw_batch(cfg, n, processes)
