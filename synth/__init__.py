"""Seeded synthetic inputs: greyscale test images, random masks, serving traces.

This module holds no part of the inpainting method. It only draws the inputs
that both the CPU oracle and the GPU path consume, so the two see identical
data. The paper measures on natural photographs (Section 5) that are not
available here; these piecewise-smooth images with step edges stand in for them
at the paper's sizes and mask densities.

Image recipe (all draws from ``numpy.random.default_rng([seed, 0])``, in this
order):

* base value 128;
* ``bumps`` Gaussian bumps, each drawing cx ~ U[0, W), cy ~ U[0, H),
  A ~ U[-80, 80], sigma ~ U[sigma_lo, sigma_hi]; the bump adds
  A * gx(x) * gy(y) with gx(x) = exp(-(x - cx)^2 / (2 sigma^2)) (gy likewise),
  evaluated at integer pixel coordinates inside the window
  |x - cx| <= 6 sigma, |y - cy| <= 6 sigma (outside it the bump is below
  1.3e-6 grey levels and is dropped);
* ``edges`` half-plane steps, each drawing px ~ U[0, W), py ~ U[0, H),
  theta ~ U[0, 2 pi), and a sign (+1 or -1, from ``rng.integers(0, 2)``); it
  adds sign * 40 at pixels where (x - px) cos(theta) + (y - py) sin(theta) > 0;
* i.i.d. Gaussian noise with standard deviation ``noise_std`` (default 2);
* clip to [0, 255] and round half to even to uint8.

Pixel (r, c) has x = c and y = r. Images are row-major, index r * W + c.

Masks draw ``k = count_from_density(density, P)`` distinct pixels uniformly
without replacement from ``default_rng([seed, 1])`` and return them sorted.

Unknown vertices of the Delaunay mesh (``make_unknowns``) are non-mask
pixels drawn uniformly without replacement from ``default_rng([seed, 4])``.

Colour images (``make_image_rgb``) share one luminance layout across their
three channels, as natural photographs do: the grey image of the same seed
(before its noise and quantisation) is the common part; channel c adds, from
``default_rng([seed, 3, c])``, ``max(1, bumps // 4)`` broad chroma bumps
(A ~ U[-50, 50], sigma ~ U[4 sigma_lo, 4 sigma_hi], same window rule) and its
own N(0, noise_std) noise, then is clipped and rounded like the grey image.
The result is planar: shape (3, H, W), channel c at [c].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "count_from_density",
    "make_image",
    "make_image_rgb",
    "make_mask",
    "make_unknowns",
    "Workload",
    "WORKLOADS",
    "serving_trace",
    "ServingRequest",
]


def count_from_density(density: float, P: int) -> int:
    """Number of mask pixels for a density: round half up of density * P.

    5% of 4096 gives 205 and 4% of 262144 gives 10486.
    """
    return int(math.floor(density * P + 0.5))


def _halfplane_add(img: np.ndarray, px: float, py: float, theta: float, amount: float) -> None:
    """Add ``amount`` where (x - px) cos(theta) + (y - py) sin(theta) > 0.

    For a fixed row the left side is monotone in x in floating point (a
    subtraction, a product by a constant and an addition of a constant are all
    monotone), so the set is a prefix or a suffix of the row. A vectorised
    bisection over rows finds the exact boundary, evaluating the expression
    with the same operations as the direct test; ``_halfplane_direct`` is the
    direct form used to check this on small images.
    """
    H, W = img.shape
    c = math.cos(theta)
    s = math.sin(theta)
    ys = np.arange(H, dtype=np.float64)
    dy = (ys - py) * s

    def cond(xi: np.ndarray) -> np.ndarray:
        return (xi.astype(np.float64) - px) * c + dy > 0

    if c == 0.0:
        rows = dy > 0
        img[rows, :] += amount
        return
    # Find t(y) = first x in [0, W] at which the row changes state.
    lo = np.zeros(H, dtype=np.int64)
    hi = np.full(H, W, dtype=np.int64)
    if c > 0:
        # cond false then true: find smallest x with cond true.
        while np.any(lo < hi):
            mid = (lo + hi) // 2
            ok = cond(mid) & (lo < hi)
            hi = np.where(ok, mid, hi)
            lo = np.where(ok | (lo >= hi), lo, mid + 1)
        for r in range(H):
            if lo[r] < W:
                img[r, lo[r]:] += amount
    else:
        # cond true then false: find smallest x with cond false.
        while np.any(lo < hi):
            mid = (lo + hi) // 2
            bad = (~cond(mid)) & (lo < hi)
            hi = np.where(bad, mid, hi)
            lo = np.where(bad | (lo >= hi), lo, mid + 1)
        for r in range(H):
            if lo[r] > 0:
                img[r, :lo[r]] += amount


def _halfplane_direct(img: np.ndarray, px: float, py: float, theta: float, amount: float) -> None:
    H, W = img.shape
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img[((x - px) * math.cos(theta) + (y - py) * math.sin(theta)) > 0] += amount


def _add_bumps(img: np.ndarray, rng, bumps: int, amp: float, sigma_lo: float,
               sigma_hi: float) -> None:
    H, W = img.shape
    for _ in range(bumps):
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        A = rng.uniform(-amp, amp)
        sig = rng.uniform(sigma_lo, sigma_hi)
        rad = 6.0 * sig
        x0 = max(0, int(math.ceil(cx - rad)))
        x1 = min(W - 1, int(math.floor(cx + rad)))
        y0 = max(0, int(math.ceil(cy - rad)))
        y1 = min(H - 1, int(math.floor(cy + rad)))
        if x0 > x1 or y0 > y1:
            continue
        xs = np.arange(x0, x1 + 1, dtype=np.float64)
        ys = np.arange(y0, y1 + 1, dtype=np.float64)
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * sig * sig))
        gy = np.exp(-((ys - cy) ** 2) / (2.0 * sig * sig))
        img[y0:y1 + 1, x0:x1 + 1] += A * np.outer(gy, gx)


def make_image(seed: int, W: int, H: int | None = None, bumps: int = 8, edges: int = 3,
               sigma_lo: float = 3.0, sigma_hi: float = 15.0, noise_std: float = 2.0,
               _direct_edges: bool = False, _field: bool = False) -> np.ndarray:
    """Synthetic 8-bit greyscale image, shape (H, W), dtype uint8 (recipe above).
    ``_field``: return the float64 image before noise, clipping and rounding."""
    if H is None:
        H = W
    rng = np.random.default_rng([seed, 0])
    img = np.full((H, W), 128.0, dtype=np.float64)
    _add_bumps(img, rng, bumps, 80.0, sigma_lo, sigma_hi)
    for _ in range(edges):
        px = rng.uniform(0.0, W)
        py = rng.uniform(0.0, H)
        theta = rng.uniform(0.0, 2.0 * math.pi)
        sign = 1.0 if rng.integers(0, 2) == 1 else -1.0
        if _direct_edges:
            _halfplane_direct(img, px, py, theta, 40.0 * sign)
        else:
            _halfplane_add(img, px, py, theta, 40.0 * sign)
    if _field:
        return img
    if noise_std > 0:
        img += rng.normal(0.0, noise_std, size=(H, W))
    np.clip(img, 0.0, 255.0, out=img)
    return np.rint(img).astype(np.uint8)


def make_image_rgb(seed: int, W: int, H: int | None = None, bumps: int = 8, edges: int = 3,
                   sigma_lo: float = 3.0, sigma_hi: float = 15.0,
                   noise_std: float = 2.0) -> np.ndarray:
    """Synthetic 8-bit colour image, planar shape (3, H, W), dtype uint8
    (recipe above)."""
    if H is None:
        H = W
    base = make_image(seed, W, H, bumps, edges, sigma_lo, sigma_hi, _field=True)
    out = np.empty((3, H, W), dtype=np.uint8)
    for c in range(3):
        rng = np.random.default_rng([seed, 3, c])
        img = base.copy()
        _add_bumps(img, rng, max(1, bumps // 4), 50.0, 4.0 * sigma_lo, 4.0 * sigma_hi)
        if noise_std > 0:
            img += rng.normal(0.0, noise_std, size=(H, W))
        np.clip(img, 0.0, 255.0, out=img)
        out[c] = np.rint(img).astype(np.uint8)
    return out


def make_mask(seed: int, P: int, density: float | None = None, k: int | None = None) -> np.ndarray:
    """Sorted, distinct int32 linear pixel indices drawn uniformly without replacement."""
    if k is None:
        if density is None:
            raise ValueError("give density or k")
        k = count_from_density(density, P)
    if not 0 <= k <= P:
        raise ValueError("mask size out of range")
    rng = np.random.default_rng([seed, 1])
    idx = rng.choice(P, size=k, replace=False)
    return np.sort(idx).astype(np.int32)


def make_unknowns(seed: int, P: int, mask_idx, count: int) -> np.ndarray:
    """Unknown vertices of the paper's Delaunay mesh: ``count`` distinct
    non-mask pixels drawn uniformly without replacement from
    ``default_rng([seed, 4])``, sorted int32."""
    mask = np.asarray(mask_idx, dtype=np.int64)
    free = np.setdiff1d(np.arange(P, dtype=np.int64), mask, assume_unique=False)
    if not 0 <= count <= free.size:
        raise ValueError("unknown-vertex count out of range")
    rng = np.random.default_rng([seed, 4])
    return np.sort(rng.choice(free, size=count, replace=False)).astype(np.int32)


@dataclass(frozen=True)
class Workload:
    """One named synthetic workload: image recipe plus mask density."""
    name: str
    seed: int
    side: int
    bumps: int
    edges: int
    sigma_lo: float
    sigma_hi: float
    density: float

    def image(self) -> np.ndarray:
        return make_image(self.seed, self.side, self.side, self.bumps, self.edges,
                          self.sigma_lo, self.sigma_hi)

    def mask(self) -> np.ndarray:
        return make_mask(self.seed, self.side * self.side, self.density)


# The five workloads: plain FP64 64^2 at 5%; mixed precision and tonal
# optimisation at 512^2 and 4%; the error-driven mask loop at 1024^2 starting
# from 1%; the large 8192^2 image at 2% (serving requests are drawn by
# ``serving_trace``).
WORKLOADS = {
    "plain64": Workload("plain64", 1, 64, 8, 3, 3.0, 15.0, 0.05),
    "tonal512": Workload("tonal512", 2, 512, 32, 8, 3.0, 15.0, 0.04),
    "densify1024": Workload("densify1024", 3, 1024, 64, 16, 3.0, 15.0, 0.01),
    "large8192": Workload("large8192", 5, 8192, 4096, 256, 5.0, 60.0, 0.02),
}


@dataclass(frozen=True)
class ServingRequest:
    index: int
    arrival_s: float
    side: int
    density: float
    image_seed: int

    @property
    def bumps(self) -> int:
        return max(8, self.side // 16)

    @property
    def edges(self) -> int:
        return max(3, self.side // 64)

    def image(self) -> np.ndarray:
        return make_image(self.image_seed, self.side, self.side, self.bumps, self.edges)

    def mask(self) -> np.ndarray:
        return make_mask(self.image_seed, self.side * self.side, self.density)


def serving_trace(seed: int = 4, n: int = 256, rate_hz: float = 4.0,
                  sides=(128, 256, 512, 1024, 2048), dens_lo: float = 0.02,
                  dens_hi: float = 0.10) -> list[ServingRequest]:
    """Poisson arrivals at ``rate_hz``; side uniform over ``sides``; density U[lo, hi].

    Draws from ``default_rng([seed, 2])``: per request, an exponential
    inter-arrival gap, then the side, then the density. Request i uses image
    seed 1000 + i.
    """
    rng = np.random.default_rng([seed, 2])
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        side = int(sides[int(rng.integers(0, len(sides)))])
        dens = float(rng.uniform(dens_lo, dens_hi))
        out.append(ServingRequest(i, t, side, dens, 1000 + i))
    return out


def busiest_block(img: np.ndarray, block: int) -> tuple[int, int]:
    """(row, col) origin of the block-aligned square with the most pixels
    strictly between 0 and 255 (ties: the first in row-major order)."""
    H, W = img.shape
    best, arg = -1, (0, 0)
    for r in range(0, H - block + 1, block):
        for c in range(0, W - block + 1, block):
            t = img[r:r + block, c:c + block]
            cnt = int(np.count_nonzero((t > 0) & (t < 255)))
            if cnt > best:
                best, arg = cnt, (r, c)
    return arg


def crop(img: np.ndarray, mask_idx: np.ndarray, r0: int, c0: int, side: int):
    """The side x side crop at (r0, c0) of an image and of its mask (mask
    indices re-numbered within the crop, ascending)."""
    W = img.shape[1]
    rows = np.asarray(mask_idx, dtype=np.int64) // W
    cols = np.asarray(mask_idx, dtype=np.int64) % W
    sel = (rows >= r0) & (rows < r0 + side) & (cols >= c0) & (cols < c0 + side)
    m = ((rows[sel] - r0) * side + (cols[sel] - c0)).astype(np.int32)
    return np.ascontiguousarray(img[r0:r0 + side, c0:c0 + side]), np.sort(m)
