"""Seeded synthetic particle-image pairs with a known displacement field.

The renderer follows the paper's in-house generator conventions (section
"Homogeneous Isotropic Turbulence", synthetic-image paragraph): particles are
Gaussian blobs whose size is given by the full width at half maximum,
FWHM = 2 sqrt(2 ln 2) sigma.  We add what that paragraph leaves open:

* pixel-integrated blobs: a pixel centred at integer (i, j) receives
  A * E(i - x_p) * E(j - y_p), where E is the pixel average of
  exp(-t^2 / (2 sigma^2)) over [t - 1/2, t + 1/2], written with erf and
  normalised to E(0) = 1, truncated at 4 sigma + 1 px;
* midpoint-symmetric advection: a particle whose midpoint position is p sits
  at p - d(p)/2 in frame 0 and at p + d(p)/2 in frame 1, so the ground truth
  at pixel m is d(m) exactly (consistent with the midpoint warps of the
  symmetric SSD objective, Eq. of_symmetric);
* peak amplitude A ~ U(amp_lo, amp_hi) * full scale, zero background,
  additive Gaussian noise, rounding to the nearest integer and clipping to
  [0, 2^B - 1] for integer frames.

This module draws random numbers and renders images.  It holds none of the
estimator's arithmetic and is shared, as an input generator only, by the
oracle tests, the GPU tests and the benchmark.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional, Tuple

import numpy as np
from scipy.special import erf

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))  # 2.35482...

FlowFn = Callable[[np.ndarray, np.ndarray], Tuple[np.ndarray, np.ndarray]]


@dataclass
class ParticlePair:
    frame0: np.ndarray          # [H, W], uint8 / uint16 / float32
    frame1: np.ndarray
    gt: np.ndarray              # [2, H, W] float64 ground-truth displacement (u, v) in px/frame
    bit_depth: int              # 8 / 12 / 16 for integer frames, 0 for float frames
    n_particles: int


def _pixel_profile(t: np.ndarray, sigma: float) -> np.ndarray:
    """Pixel-averaged Gaussian profile, normalised to 1 at t = 0."""
    c = sigma * math.sqrt(2.0)
    e = erf((t + 0.5) / c) - erf((t - 0.5) / c)
    return e / (2.0 * erf(0.5 / c))


def render_particles(h: int, w: int, xs: np.ndarray, ys: np.ndarray, amps: np.ndarray,
                     sigma: float, chunk: int = 200_000) -> np.ndarray:
    """Render pixel-integrated Gaussian blobs into a float64 [h, w] image."""
    img = np.zeros(h * w, dtype=np.float64)
    half = int(math.ceil(4.0 * sigma + 1.0))
    offs = np.arange(-half, half + 1)
    for s in range(0, xs.size, chunk):
        x = xs[s:s + chunk]
        y = ys[s:s + chunk]
        a = amps[s:s + chunk]
        cx = np.rint(x).astype(np.int64)
        cy = np.rint(y).astype(np.int64)
        px = cx[:, None] + offs[None, :]                  # [n, k] column indices
        py = cy[:, None] + offs[None, :]                  # [n, k] row indices
        ex = _pixel_profile(px - x[:, None], sigma)        # [n, k]
        ey = _pixel_profile(py - y[:, None], sigma) * a[:, None]
        okx = (px >= 0) & (px < w)
        oky = (py >= 0) & (py < h)
        vals = ey[:, :, None] * ex[:, None, :]             # [n, ky, kx]
        ok = oky[:, :, None] & okx[:, None, :]
        idx = py[:, :, None] * w + px[:, None, :]
        img += np.bincount(idx[ok], weights=vals[ok], minlength=h * w)
    return img.reshape(h, w)


def _quantise(img: np.ndarray, bit_depth: int, rng: np.random.Generator,
              noise_sigma: float, container: np.dtype) -> np.ndarray:
    full = float(2 ** bit_depth - 1)
    if noise_sigma > 0:
        img = img + rng.normal(0.0, noise_sigma, size=img.shape)
    return np.clip(np.rint(img), 0.0, full).astype(container)


def make_pair(h: int, w: int, flow: FlowFn, *, fwhm: float, ppp: float, seed: int,
              bit_depth: int = 8, noise: float = 0.0, amp: Tuple[float, float] = (0.5, 1.0),
              max_disp: Optional[float] = None) -> ParticlePair:
    """Render one image pair advected by ``flow``.

    ``flow(x, y)`` returns the displacement (dx, dy) in px/frame at midpoint
    positions (x along columns, y along rows, pixel centres at integers).
    ``bit_depth`` 0 gives float32 frames in [0, 1] with ``noise`` in intensity
    units; otherwise integer frames (uint8 for 8 bit, uint16 for 12/16 bit,
    right-aligned) with ``noise`` in digital numbers.
    """
    rng = np.random.default_rng(seed)
    sigma = fwhm / FWHM_PER_SIGMA
    if hasattr(flow, "grid"):
        du, dv = flow.grid(h, w)
    else:
        gy, gx = np.mgrid[0:h, 0:w].astype(np.float64)
        du, dv = flow(gx, gy)
    gt = np.stack([np.broadcast_to(du, (h, w)), np.broadcast_to(dv, (h, w))]).astype(np.float64)
    if max_disp is None:
        max_disp = float(np.max(np.hypot(gt[0], gt[1]))) if gt.size else 0.0
    margin = math.ceil(max_disp) + 4.0 * sigma + 2.0
    ext_w, ext_h = w + 2 * margin, h + 2 * margin
    n = int(round(ppp * ext_w * ext_h))
    px = rng.uniform(-margin - 0.5, w - 0.5 + margin, size=n)
    py = rng.uniform(-margin - 0.5, h - 0.5 + margin, size=n)
    full = 1.0 if bit_depth == 0 else float(2 ** bit_depth - 1)
    amps = rng.uniform(amp[0], amp[1], size=n) * full
    if hasattr(flow, "inside"):
        keep = ~flow.inside(px, py)
        px, py, amps = px[keep], py[keep], amps[keep]
        n = int(px.size)
    dx, dy = flow(px, py)
    dx = np.broadcast_to(dx, px.shape)
    dy = np.broadcast_to(dy, py.shape)
    img0 = render_particles(h, w, px - 0.5 * dx, py - 0.5 * dy, amps, sigma)
    img1 = render_particles(h, w, px + 0.5 * dx, py + 0.5 * dy, amps, sigma)
    if bit_depth == 0:
        if noise > 0:
            img0 = img0 + rng.normal(0.0, noise, size=img0.shape)
            img1 = img1 + rng.normal(0.0, noise, size=img1.shape)
        f0 = img0.astype(np.float32)
        f1 = img1.astype(np.float32)
    else:
        container = np.uint8 if bit_depth <= 8 else np.uint16
        f0 = _quantise(img0, bit_depth, rng, noise, container)
        f1 = _quantise(img1, bit_depth, rng, noise, container)
    return ParticlePair(f0, f1, gt, bit_depth, n)


def make_texture(h: int, w: int, *, fwhm: float, ppp: float, seed: int,
                 margin: int = 0) -> np.ndarray:
    """Float64 particle texture of size [h + 2 margin, w + 2 margin] (no noise).

    Used to build exactly shifted pairs: cropping one texture at two integer
    offsets gives frames related by an exact integer translation.
    """
    rng = np.random.default_rng(seed)
    sigma = fwhm / FWHM_PER_SIGMA
    hh, ww = h + 2 * margin, w + 2 * margin
    n = int(round(ppp * hh * ww))
    px = rng.uniform(-0.5, ww - 0.5, size=n)
    py = rng.uniform(-0.5, hh - 0.5, size=n)
    amps = rng.uniform(0.5, 1.0, size=n)
    return render_particles(hh, ww, px, py, amps, sigma)


def make_stripes_pair(h: int, w: int, tx: float, ty: float, *, seed: int, noise: float = 0.5,
                      fwhm: float = 2.5, density: float = 0.35) -> ParticlePair:
    """An aperture-problem pair: a one-dimensional particle texture along s = x + y (oblique
    stripes of Gaussian line profiles, FWHM ``fwhm`` across the stripe, ``density`` lines per unit
    of s), translated by (tx, ty) between the frames, 8-bit with Gaussian noise of ``noise`` DN.
    Only the component of the motion along (1, 1) is visible in such images; the window normal
    matrices are then nearly singular at most pixels.  The ground truth is the translation."""
    rng = np.random.default_rng(seed)
    smin, smax = -40.0, float(h + w) + 40.0
    n = int(density * (smax - smin))
    s0 = rng.uniform(smin, smax, n)
    amps = rng.uniform(0.5, 1.0, n)
    # FWHM measured across the stripes (along (1, 1) / sqrt(2)) is fwhm; in units of s it is sqrt(2) fwhm
    sig = fwhm / FWHM_PER_SIGMA * math.sqrt(2.0)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    frames = []
    for sgn in (-0.5, 0.5):
        s = xx + yy - sgn * (tx + ty)
        img = np.zeros((h, w))
        for c, a in zip(s0, amps):
            img += a * np.exp(-0.5 * ((s - c) / sig) ** 2)
        img = 255.0 * img / 1.2 + noise * rng.normal(size=(h, w))
        frames.append(np.clip(np.round(img), 0, 255).astype(np.uint8))
    gt = np.stack([np.full((h, w), float(tx)), np.full((h, w), float(ty))])
    return ParticlePair(frames[0], frames[1], gt, 8, n)
