"""Seeded synthetic pairs (grayscale, float32 in roughly [0, 1]).

Each generator returns a dict with ``img1`` (H x W), ``img2`` (H' x W'),
optionally ``flow`` (a callable mapping source pixel coordinates to the true
target coordinates) and ``meta`` (seed, sizes, recipe).  Every random number
comes from ``numpy.random.default_rng(seed)`` in a fixed draw order, so the
same call gives the same pair on any machine with the same numpy.

Recipes (the stand-ins for the paper's movie and driving frames):

* ``c1``  64x64, seed 101: white noise blurred with sigma 1.5 and min-max
  scaled; image 2 is image 1 shifted by (+5, -3) px with reflected borders,
  plus N(0, 0.02^2) noise.  A source point p appears at p + (5, -3).
* ``c2``  256x192, seed 202: four-octave blurred-noise texture with one
  rectangle of 20 % of the area replaced by a tiled 8x8 random pattern
  (period 8 px); image 2 is image 1 warped by a smooth random field (white
  noise blurred with sigma 24, scaled to a max norm of 20 px) plus noise.
* ``c3``  512x256, seed 303: c1-style content, c2-style field with max 40 px,
  a brightness gain drawn from U[0.8, 1.2] on image 2, plus noise.
* ``c4``  256x192, seed 404: c1-style content shifted by (+5, -3).
* ``c5``  32 pairs, seeds 5000+j: W ~ U{128..621}, H ~ U{96..188}, c1-style
  content, c2-style field with max 30 px.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

NOISE_SIGMA = 0.02


def _minmax(a: np.ndarray) -> np.ndarray:
    lo, hi = a.min(), a.max()
    return (a - lo) / (hi - lo)


def _reflect_index(i: np.ndarray, n: int) -> np.ndarray:
    """Half-sample symmetric reflection of integer indices into [0, n)."""
    i = np.mod(i, 2 * n)
    return np.where(i >= n, 2 * n - 1 - i, i)


def blurred_noise(rng, h: int, w: int, sigma: float = 1.5) -> np.ndarray:
    """White noise blurred with a Gaussian (reflect border), min-max scaled."""
    z = rng.standard_normal((h, w))
    return _minmax(ndimage.gaussian_filter(z, sigma, mode="reflect"))


def multi_octave_texture(rng, h: int, w: int, octaves: int = 4) -> np.ndarray:
    acc = np.zeros((h, w))
    for k in range(octaves):
        z = ndimage.gaussian_filter(rng.standard_normal((h, w)), 2.0 ** k, mode="reflect")
        acc += 2.0 ** (-k) * (z - z.mean()) / z.std()
    return _minmax(acc)


def smooth_field(rng, h: int, w: int, max_disp: float, sigma: float = 24.0) -> np.ndarray:
    """Smooth displacement field D (2 x h x w, [dx, dy]) with max |D| = max_disp."""
    d = np.stack([ndimage.gaussian_filter(rng.standard_normal((h, w)), sigma, mode="reflect")
                  for _ in range(2)])
    norm = np.sqrt((d ** 2).sum(0)).max()
    return d * (max_disp / norm)


def _bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    h, w = img.shape[:2]
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0
    xa, xb = _reflect_index(x0, w), _reflect_index(x0 + 1, w)
    ya, yb = _reflect_index(y0, h), _reflect_index(y0 + 1, h)
    return ((1 - fy) * ((1 - fx) * img[ya, xa] + fx * img[ya, xb])
            + fy * ((1 - fx) * img[yb, xa] + fx * img[yb, xb]))


def warp_bilinear(img: np.ndarray, field: np.ndarray) -> np.ndarray:
    """out(y) = img(y - D(y)), bilinear with reflected borders."""
    h, w = img.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    return _bilinear(img, xx - field[0], yy - field[1])


def shift_reflect(img: np.ndarray, dx: int, dy: int) -> np.ndarray:
    """out(x, y) = img(x - dx, y - dy) with reflected borders."""
    h, w = img.shape
    ys = _reflect_index(np.arange(h) - dy, h)
    xs = _reflect_index(np.arange(w) - dx, w)
    return img[np.ix_(ys, xs)]


def invert_field(field: np.ndarray, px: np.ndarray, py: np.ndarray, iters: int = 50):
    """Target position p' of source points p for a warp out(y) = in(y - D(y)).

    Solves p' = p + D(p') by fixed-point iteration (D is smooth and small)."""
    qx, qy = px.astype(np.float64), py.astype(np.float64)
    for _ in range(iters):
        qx = px + _bilinear(field[0], qx, qy)
        qy = py + _bilinear(field[1], qx, qy)
    return qx, qy


def _finish(rng, img2: np.ndarray) -> np.ndarray:
    return img2 + rng.normal(0.0, NOISE_SIGMA, img2.shape)


def _shift_pair(seed: int, w: int, h: int, shift=(5, -3)):
    rng = np.random.default_rng(seed)
    i1 = blurred_noise(rng, h, w, 1.5)
    i2 = _finish(rng, shift_reflect(i1, *shift))
    sx, sy = shift

    def flow(px, py):
        return np.asarray(px, np.float64) + sx, np.asarray(py, np.float64) + sy

    meta = dict(seed=seed, W=w, H=h, kind="shift", shift=list(shift), noise=NOISE_SIGMA)
    return dict(img1=i1.astype(np.float32), img2=i2.astype(np.float32), flow=flow, meta=meta)


def _warp_pair(seed: int, w: int, h: int, max_disp: float, texture: str, gain: bool,
               rng=None):
    rng = np.random.default_rng(seed) if rng is None else rng
    if texture == "octaves":
        i1 = multi_octave_texture(rng, h, w)
        rw, rh = int(round(w * np.sqrt(0.2))), int(round(h * np.sqrt(0.2)))
        x0 = int(rng.integers(0, w - rw + 1))
        y0 = int(rng.integers(0, h - rh + 1))
        tile = rng.random((8, 8))
        ty, tx = np.mgrid[0:rh, 0:rw]
        i1[y0:y0 + rh, x0:x0 + rw] = tile[ty % 8, tx % 8]
        extra = dict(periodic_rect=[x0, y0, rw, rh])
    else:
        i1 = blurred_noise(rng, h, w, 1.5)
        extra = {}
    field = smooth_field(rng, h, w, max_disp)
    i2 = warp_bilinear(i1, field)
    g = 1.0
    if gain:
        g = float(rng.uniform(0.8, 1.2))
        i2 = i2 * g
    i2 = _finish(rng, i2)

    def flow(px, py):
        return invert_field(field, np.asarray(px, np.float64), np.asarray(py, np.float64))

    meta = dict(seed=seed, W=w, H=h, kind="warp", max_disp=max_disp, texture=texture,
                gain=g, noise=NOISE_SIGMA, **extra)
    return dict(img1=i1.astype(np.float32), img2=i2.astype(np.float32), flow=flow, meta=meta)


CONFIGS = {
    "c1": lambda: _shift_pair(101, 64, 64),
    "c2": lambda: _warp_pair(202, 256, 192, 20.0, "octaves", gain=False),
    "c3": lambda: _warp_pair(303, 512, 256, 40.0, "noise", gain=True),
    "c4": lambda: _shift_pair(404, 256, 192),
}

# Pyramid tops fixed by the workloads (0 = the default rule of the pyramid loop).
CONFIG_NMAX = {"c1": 32, "c2": 64, "c3": 0, "c4": 0}


def make_pair(name: str):
    return CONFIGS[name]()


def make_batch(n: int = 32, base_seed: int = 5000, max_disp: float = 30.0):
    """Uneven-size pairs for batched runs: W ~ U{128..621}, H ~ U{96..188}."""
    out = []
    for j in range(n):
        rng = np.random.default_rng(base_seed + j)
        w = int(rng.integers(128, 622))
        h = int(rng.integers(96, 189))
        out.append(_warp_pair(base_seed + j, w, h, max_disp, "noise", gain=False, rng=rng))
    return out


def make_warp_pair(seed: int, w: int, h: int, max_disp: float = 30.0) -> dict:
    """One pair of the uneven-batch recipe at a chosen size: c1-style content
    warped by a smooth field of the given maximum displacement, plus noise."""
    return _warp_pair(seed, w, h, max_disp, "noise", gain=False)


def sub_pair(pair: dict, x0: int, y0: int, w: int, h: int) -> dict:
    """Crop both images of a pair to the same window."""
    return dict(img1=np.ascontiguousarray(pair["img1"][y0:y0 + h, x0:x0 + w]),
                img2=np.ascontiguousarray(pair["img2"][y0:y0 + h, x0:x0 + w]),
                meta=dict(pair["meta"], crop=[x0, y0, w, h]))
