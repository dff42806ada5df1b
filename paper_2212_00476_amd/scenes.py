"""Seeded synthetic stereo scenes.

These stand in for the rectified KITTI-2015-sized grayscale pairs the paper
evaluates on (Sec. V: 1280x384 and ~1242x375, D = 128), which are not
available here.  A scene is a stack of planar layers rendered exactly into both
views: layer k has a region on the reference (left) grid, a disparity plane
d_k(x, y) = a + b x + c y and its own texture.  The left view shows the
frontmost layer (largest disparity); the right view places each layer's texture
at x' = x - d_k(x, y), inverted in closed form, with gain, bias and Gaussian
noise, rounded half-to-even and clipped to 0..255.  Right pixels with no
preimage get fresh noise.  Ground truth is d_top on the left grid, with a
validity mask that drops occluded pixels and targets outside the frame.

This module computes no part of the matching method; it only makes inputs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class StereoPair:
    left: np.ndarray       # uint8 [H][W], reference image
    right: np.ndarray      # uint8 [H][W], target image
    gt: np.ndarray         # float32 [H][W], ground-truth disparity on the left grid
    valid: np.ndarray      # bool [H][W]
    max_disp: int
    seed: int


def _box3(img):
    p = np.pad(img, 1, mode="edge")
    out = np.zeros_like(img, dtype=np.float64)
    for j in range(3):
        for i in range(3):
            out += p[j:j + img.shape[0], i:i + img.shape[1]]
    return out / 9.0


def _blur(img, passes):
    for _ in range(passes):
        img = _box3(img)
    return img


def _octave_texture(rng, H, W, std=40.0):
    """Multi-octave blurred noise, mean 128, the given standard deviation."""
    acc = np.zeros((H, W))
    for k, amp in enumerate((1.0, 0.7, 0.5, 0.35)):
        step = 2 ** k
        h, w = (H + step - 1) // step + 2, (W + step - 1) // step + 2
        n = rng.standard_normal((h, w))
        n = np.repeat(np.repeat(n, step, axis=0), step, axis=1)[:H, :W]
        acc += amp * _blur(n, 1 + k // 2)
    acc = (acc - acc.mean()) / max(acc.std(), 1e-9)
    return 128.0 + std * acc


@dataclass
class _Layer:
    a: float
    b: float
    c: float
    tex: np.ndarray        # float64 texture; entry [j][i] is pixel (ox + i, oy + j), sampled at fractional x
    inside: callable       # (x, y) float arrays -> bool array
    ox: int = 0
    oy: int = 0


def _in_box(fn, xlo, xhi, ylo, yhi):
    """`fn` evaluated only at the points inside its bounding box (False outside)."""
    def inside(x, y):
        m = (x >= xlo) & (x <= xhi) & (y >= ylo) & (y <= yhi)
        out = np.zeros(np.shape(x), bool)
        out[m] = fn(x[m], y[m])
        return out
    return inside


def _sample(L, x, y):
    """Linear interpolation of a layer's texture along x at fractional x (integer rows y)."""
    W = L.tex.shape[1]
    x = np.clip(x - L.ox, 0.0, W - 1.000001)
    x0 = np.floor(x).astype(np.int64)
    f = x - x0
    y = np.clip(y - L.oy, 0, L.tex.shape[0] - 1)
    return L.tex[y, x0] * (1.0 - f) + L.tex[y, x0 + 1] * f


def _render(layers, H, W, D, rng, gain, bias, noise, seed):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    yi = ys.astype(np.int64)
    # left view: frontmost layer on the left grid
    top = np.full((H, W), -1, np.int64)
    dtop = np.full((H, W), -np.inf)
    for k, L in enumerate(layers):
        dk = L.a + L.b * xs + L.c * ys
        m = L.inside(xs, ys) & (dk > dtop)
        top[m] = k
        dtop[m] = dk[m]
    left = np.empty((H, W))
    for k, L in enumerate(layers):
        m = top == k
        left[m] = L.tex[yi[m] - L.oy, xs[m].astype(np.int64) - L.ox]
    # right view: at x', the layer whose preimage x = (x' + a + c y) / (1 - b) is frontmost
    rtop = np.full((H, W), -1, np.int64)
    rd = np.full((H, W), -np.inf)
    rx = np.zeros((H, W))
    for k, L in enumerate(layers):
        x = (xs + L.a + L.c * ys) / (1.0 - L.b)
        ok = (x >= 0.0) & (x <= W - 1) & L.inside(x, ys)
        dk = x - xs
        m = ok & (dk > rd)
        rtop[m] = k
        rd[m] = dk[m]
        rx[m] = x[m]
    right = rng.uniform(0.0, 255.0, (H, W))
    for k, L in enumerate(layers):
        m = rtop == k
        right[m] = gain * _sample(L, rx[m], yi[m]) + bias
    right = right + rng.normal(0.0, noise, (H, W))
    right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    left = np.clip(np.rint(left), 0, 255).astype(np.uint8)
    # validity: target inside the frame, not occluded in the right view, disparity in range
    xt = xs - dtop
    valid = (xt >= 0.0) & (dtop >= 0.0) & (dtop <= D - 1)
    for k, L in enumerate(layers):
        x = (xt + L.a + L.c * ys) / (1.0 - L.b)
        occ = (x >= 0.0) & (x <= W - 1) & L.inside(x, ys) & ((x - xt) > dtop + 1e-6) & (top != k)
        valid &= ~occ
    return StereoPair(left=left, right=right, gt=dtop.astype(np.float32), valid=valid, max_disp=D, seed=seed)


def bands_pair(W=320, H=96, D=32, seed=0, band_disps=(5, 12, 20), gain=0.9, bias=5.0, noise=2.0):
    """Piecewise-constant disparity: vertical bands of equal width sharing one
    texture (uniform 0..255 noise, box-blurred 3x3)."""
    rng = np.random.default_rng(seed)
    tex = _box3(rng.uniform(0.0, 255.0, (H, W + 2)))
    n = len(band_disps)
    edges = [round(i * W / n) for i in range(n + 1)]
    layers = []
    for k, d in enumerate(band_disps):
        lo, hi = edges[k], edges[k + 1]
        layers.append(_Layer(a=float(d), b=0.0, c=0.0, tex=tex,
                             inside=(lambda lo, hi: lambda x, y: (x >= lo) & (x < hi))(lo, hi)))
    pair = _render(layers, H, W, D, rng, gain, bias, noise, seed)
    pair.band_edges = edges
    pair.band_disps = tuple(band_disps)
    return pair


def _ellipse(cx, cy, rx, ry):
    return lambda x, y: ((x - cx) / rx) ** 2 + ((y - cy) / ry) ** 2 <= 1.0


def _convex_quad(pts):
    pts = np.asarray(pts, np.float64)
    c = pts.mean(axis=0)
    ang = np.arctan2(pts[:, 1] - c[1], pts[:, 0] - c[0])
    pts = pts[np.argsort(ang)]

    def inside(x, y):
        ok = np.ones(np.shape(x), bool)
        for i in range(4):
            x0, y0 = pts[i]
            x1, y1 = pts[(i + 1) % 4]
            ok &= (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0) >= 0.0
        return ok
    return inside


def planes_pair(W=1280, H=384, D=128, seed=1, n_planes=None, noise=2.0):
    """Textured background with a gentle disparity slope in [0, D/8] plus
    randomly placed slanted planes (ellipses or convex quads), each with its own
    texture and |b|, |c| <= 0.2, disparity kept inside [0, D-1] over its region;
    target gain U(0.8, 1.2), bias U(-10, 10), noise sigma 2."""
    rng = np.random.default_rng(seed)
    if n_planes is None:
        n_planes = int(np.clip(round(6 * (W * H) / (1280 * 384)), 2, 24))
    layers = []
    dmax_bg = D / 8.0
    b0 = rng.uniform(0.0, 0.5) * dmax_bg / W
    c0 = (dmax_bg - b0 * W) / H * rng.uniform(0.3, 1.0)
    layers.append(_Layer(a=0.0, b=b0, c=c0, tex=_octave_texture(rng, H, W + 2),
                         inside=lambda x, y: np.ones(np.shape(x), bool)))
    for _ in range(n_planes):
        cx, cy = rng.uniform(0.1 * W, 0.9 * W), rng.uniform(0.1 * H, 0.9 * H)
        sx, sy = rng.uniform(0.05 * W, 0.18 * W), rng.uniform(0.08 * H, 0.3 * H)
        if rng.uniform() < 0.5:
            inside = _ellipse(cx, cy, sx, sy)
            xlo, xhi, ylo, yhi = cx - sx, cx + sx, cy - sy, cy + sy
        else:
            ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, 4))
            pts = np.stack([cx + sx * np.cos(ang), cy + sy * np.sin(ang)], axis=1)
            inside = _convex_quad(pts)
            xlo, xhi = pts[:, 0].min(), pts[:, 0].max()
            ylo, yhi = pts[:, 1].min(), pts[:, 1].max()
        b, c = rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2)
        corners = [b * x + c * y for x in (xlo, xhi) for y in (ylo, yhi)]
        span = max(corners) - min(corners)
        if span > D - 1:
            s = (D - 1) / span
            b, c = b * s, c * s
            corners = [b * x + c * y for x in (xlo, xhi) for y in (ylo, yhi)]
        lo, hi = -min(corners), D - 1 - max(corners)
        a = rng.uniform(min(lo + dmax_bg, hi), hi) if hi > lo else lo
        # texture and mask over the plane's bounding box only (columns one past
        # each side for the interpolation of the target view)
        ox, oy = max(0, int(np.floor(xlo)) - 1), max(0, int(np.floor(ylo)))
        tw = min(W + 2, int(np.ceil(xhi)) + 3) - ox
        th = min(H, int(np.ceil(yhi)) + 1) - oy
        tex = _octave_texture(rng, max(th, 1), max(tw, 2), std=rng.uniform(25, 50))
        layers.append(_Layer(a=a, b=b, c=c, tex=tex, inside=_in_box(inside, xlo, xhi, ylo, yhi), ox=ox, oy=oy))
    gain, bias = rng.uniform(0.8, 1.2), rng.uniform(-10.0, 10.0)
    return _render(layers, H, W, D, rng, gain, bias, noise, seed)


def cost_volume(W, H, D, seed=0, structured=True):
    """Seeded float32 cost volume [H][W][D] with values in [0, 2] (the range of
    1 - ZNCC), for aggregation tests that start from a given volume.  Plain:
    independent uniform values.  Structured: each pixel has a true disparity
    from a piecewise-planar field, and its costs grow with the distance to it,
    plus uniform noise -- a volume with the minima a matching cost has."""
    rng = np.random.default_rng(seed)
    if not structured:
        return rng.uniform(0.0, 2.0, (H, W, D)).astype(np.float32)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    true = np.zeros((H, W))
    for k in range(4):  # four planes, the later ones over vertical bands
        a, b, c = rng.uniform(0, D - 1), rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05)
        plane = np.clip(a + b * (x - W / 2) + c * (y - H / 2), 0, D - 1)
        band = (x >= k * W / 4) if k else np.ones_like(x, bool)
        true = np.where(band, plane, true)
    d = np.arange(D, dtype=np.float64)
    cost = np.minimum(2.0, 0.04 * np.abs(d[None, None, :] - true[:, :, None]))
    cost += rng.uniform(0.0, 0.3, cost.shape)
    return np.minimum(cost, 2.0).astype(np.float32)


def workload(name, seed=None):
    """The named synthetic workloads used by the tests and the benchmark."""
    if name == "bands_320x96_d32":
        return bands_pair(seed=0 if seed is None else seed)
    if name == "planes_1280x384_d128":
        return planes_pair(1280, 384, 128, seed=1 if seed is None else seed)
    if name == "planes_640x192_d64":
        return planes_pair(640, 192, 64, seed=100 if seed is None else seed)
    if name == "planes_1920x1080_d256":
        return planes_pair(1920, 1080, 256, seed=100 if seed is None else seed)
    raise KeyError(name)
