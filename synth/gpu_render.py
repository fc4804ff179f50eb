"""Device-side rendering of large seeded particle pairs (4-21 Mp frames).

Same conventions as :mod:`synth.particles` (pixel-integrated Gaussian blobs,
midpoint-symmetric advection, noise, rounding, clipping); particle positions
and amplitudes come from the same seeded NumPy generator, the flow is
evaluated at particle positions on the host, and only the scatter of the
blobs into the frames runs as torch operations on the device.  Input
generation only.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np
import torch

from .particles import FWHM_PER_SIGMA


def _profile(t: torch.Tensor, sigma: float) -> torch.Tensor:
    c = sigma * math.sqrt(2.0)
    return (torch.special.erf((t + 0.5) / c) - torch.special.erf((t - 0.5) / c)) / (2.0 * math.erf(0.5 / c))


def render_torch(h: int, w: int, xs: np.ndarray, ys: np.ndarray, amps: np.ndarray, sigma: float,
                 device: torch.device, chunk: int = 1 << 18) -> torch.Tensor:
    img = torch.zeros(h * w, dtype=torch.float32, device=device)
    half = int(math.ceil(4.0 * sigma + 1.0))
    offs = torch.arange(-half, half + 1, device=device)
    for s in range(0, xs.size, chunk):
        x = torch.as_tensor(xs[s:s + chunk], device=device, dtype=torch.float64)
        y = torch.as_tensor(ys[s:s + chunk], device=device, dtype=torch.float64)
        a = torch.as_tensor(amps[s:s + chunk], device=device, dtype=torch.float32)
        px = torch.round(x).long()[:, None] + offs[None, :]
        py = torch.round(y).long()[:, None] + offs[None, :]
        ex = _profile((px - x[:, None]).float(), sigma)
        ey = _profile((py - y[:, None]).float(), sigma) * a[:, None]
        ok = ((py >= 0) & (py < h))[:, :, None] & ((px >= 0) & (px < w))[:, None, :]
        vals = (ey[:, :, None] * ex[:, None, :])[ok]
        idx = (py[:, :, None] * w + px[:, None, :])[ok]
        img.index_add_(0, idx, vals)
    return img.view(h, w)


def make_pair_device(h: int, w: int, flow, *, fwhm: float, ppp: float, seed: int, bit_depth: int, noise: float,
                     device: torch.device, max_disp: float, with_gt: bool = False
                     ) -> Tuple[torch.Tensor, torch.Tensor, Optional[np.ndarray]]:
    """Frames (uint8 / uint16 / float32 device tensors) and, optionally, the ground truth."""
    rng = np.random.default_rng(seed)
    sigma = fwhm / FWHM_PER_SIGMA
    margin = math.ceil(max_disp) + 4.0 * sigma + 2.0
    n = int(round(ppp * (w + 2 * margin) * (h + 2 * margin)))
    px = rng.uniform(-margin - 0.5, w - 0.5 + margin, size=n)
    py = rng.uniform(-margin - 0.5, h - 0.5 + margin, size=n)
    full = 1.0 if bit_depth == 0 else float(2 ** bit_depth - 1)
    amps = rng.uniform(0.5, 1.0, size=n) * full
    if hasattr(flow, "inside"):
        keep = ~flow.inside(px, py)
        px, py, amps = px[keep], py[keep], amps[keep]
    dx, dy = flow(px, py)
    dx = np.broadcast_to(dx, px.shape)
    dy = np.broadcast_to(dy, py.shape)
    frames = []
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    for sgn in (-0.5, 0.5):
        img = render_torch(h, w, px + sgn * dx, py + sgn * dy, amps, sigma, device)
        if noise > 0:
            img = img + noise * torch.randn(img.shape, device=device, generator=gen)
        if bit_depth == 0:
            frames.append(img.contiguous())
        else:
            if bit_depth > 15:
                raise ValueError("device frames hold up to 15 significant bits (int16 containers)")
            q = torch.clamp(torch.round(img), 0, full)
            frames.append((q.to(torch.uint8) if bit_depth <= 8 else q.to(torch.int16)).contiguous())
    gt = None
    if with_gt:
        if hasattr(flow, "grid"):
            gu, gv = flow.grid(h, w)
        else:
            gy, gx = np.mgrid[0:h, 0:w].astype(np.float64)
            gu, gv = flow(gx, gy)
        gt = np.stack([np.broadcast_to(gu, (h, w)), np.broadcast_to(gv, (h, w))])
    return frames[0], frames[1], gt
