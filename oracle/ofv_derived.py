"""FP64 CPU oracle of the live derived quantities (test infrastructure).

This module is test infrastructure, not part of the product: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the HIP library.

The paper's live pipeline turns every measured velocity field into
observables while it streams (the cylinder-wake experiment of the section
on live measurements): the out-of-plane vorticity field, velocity probes at
fixed points, and the recirculation area of Eq. (RA) - the summed area of
the pixels whose streamwise velocity opposes the free stream.  Each of them
has a plain definition, written out here in float64.  Readings taken where
the paper is silent:

 R19 Vorticity in image coordinates (x along columns, y along rows, y
     pointing down) of the physical velocity (U, V) = (u dx / dt, v dz / dt),
     with u, v the displacement in pixels per frame pair, dx, dz the pixel
     size along x and y and dt the time between the frames:
         omega = dV/dX - dU/dY = ((dz / dx) dv/di - (dx / dz) du/dj) / dt.
     The per-pixel derivative d/di is the central difference
     (f[i+1] - f[i-1]) / 2 inside, the one-sided differences f[1] - f[0]
     and f[n-1] - f[n-2] at the two edges, and 0 along a dimension of one
     pixel.  Masked pixels get 0; derivatives next to a masked pixel use the
     field as estimated.  (For a y-up convention, negate.)
 R20 RA = dx dz #{unmasked pixels with s u < 0}, s = +1 when the free
     stream runs along +x and -1 along -x: the Heaviside of Eq. (RA) is 1
     for strictly negative streamwise velocity only.
 R21 A probe at (x, y) is the bilinear sample of the field with clamped
     coordinates (the interpolation of the warps, reading R7), scaled to
     (u dx / dt, v dz / dt).
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import torch

from .ofv_oracle import DT, _t, bilinear


def ddi(f: torch.Tensor) -> torch.Tensor:
    """Per-pixel derivative along columns (R19): central inside, one-sided at the edges."""
    f = _t(f)
    d = torch.zeros_like(f)
    w = f.shape[1]
    if w < 2:
        return d
    d[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / 2.0
    d[:, 0] = f[:, 1] - f[:, 0]
    d[:, -1] = f[:, -1] - f[:, -2]
    return d


def ddj(f: torch.Tensor) -> torch.Tensor:
    """Per-pixel derivative along rows (R19)."""
    return ddi(_t(f).T).T


def _valid(mask, shape) -> torch.Tensor:
    if mask is None:
        return torch.ones(shape, dtype=torch.bool)
    return torch.as_tensor(np.asarray(mask)) != 0


def vorticity(u, v, dx: float = 1.0, dz: float = 1.0, dt: float = 1.0, mask=None) -> torch.Tensor:
    """Out-of-plane vorticity of the field (R19), 0 at masked pixels."""
    u, v = _t(u), _t(v)
    om = (dz / dx) / dt * ddi(v) - (dx / dz) / dt * ddj(u)
    return torch.where(_valid(mask, u.shape), om, torch.zeros((), dtype=DT))


def recirculation_area(u, dx: float = 1.0, dz: float = 1.0, mask=None, sign: int = 1) -> Tuple[float, int]:
    """Eq. (RA) with reading R20: (area, number of pixels)."""
    u = _t(u)
    hit = (sign * u < 0) & _valid(mask, u.shape)
    n = int(hit.sum().item())
    return float(n) * float(dx) * float(dz), n


def probes(u, v, xy, dx: float = 1.0, dz: float = 1.0, dt: float = 1.0) -> torch.Tensor:
    """[n, 2] physical velocity at the probe points xy[n, 2] = (x, y) (R21)."""
    u, v = _t(u), _t(v)
    p = _t(xy).reshape(-1, 2)
    pu = bilinear(u, p[:, 0], p[:, 1]) * (dx / dt)
    pv = bilinear(v, p[:, 0], p[:, 1]) * (dz / dt)
    return torch.stack([pu, pv], dim=1)
