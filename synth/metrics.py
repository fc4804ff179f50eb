"""Accuracy of an estimated field against the analytic field of a synthetic
Rankine vortex: the profile-unfolding discrepancy Psi of Eq. (psi_metric)
and the mean endpoint error.

This is evaluation of outputs against the generator's ground truth, not
part of the estimator.  It works on torch tensors on any device so that a
parameter sweep can score thousands of fields where they were computed.

Psi (the paper's "Rankine profile-unfolding metric"): one-pixel profiles of
the displacement magnitude through the vortex centre are taken at angles
covering 180 degrees, one angle step dtheta = pi / N_theta with
r_max * dtheta ~ 1 px, and stacked into arrays R_th (theory) and R_OFV
(estimate); Psi is the summed absolute difference divided by the unfolded
area, i.e. the number of samples.  Readings where the paper is silent: the
region of interest is the disc of radius r_max = 2 R (the core radius),
capped at 0.45 of the smaller image side; samples are one pixel apart along
each profile, the estimated magnitude is interpolated bilinearly with
clamped coordinates, and the theoretical one is the exact magnitude of the
analytic field at the sample's radius.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import torch


def unfolding_grid(cx: float, cy: float, r_max: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Sample points (x, y) [n_theta, n_r] of the unfolded profiles and their signed radius."""
    n_r = 2 * int(math.floor(r_max)) + 1
    s = np.arange(n_r, dtype=np.float64) - (n_r - 1) // 2
    n_theta = max(1, int(math.ceil(math.pi * r_max)))
    th = np.arange(n_theta, dtype=np.float64) * (math.pi / n_theta)
    x = cx + np.cos(th)[:, None] * s[None, :]
    y = cy + np.sin(th)[:, None] * s[None, :]
    return x, y, np.broadcast_to(s, x.shape)


def _bilinear_many(planes: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """planes [B, H, W] sampled at the same points (x, y) with clamped coordinates."""
    _, h, w = planes.shape
    xc = torch.clamp(x, 0.0, float(w - 1))
    yc = torch.clamp(y, 0.0, float(h - 1))
    x0 = torch.floor(xc)
    y0 = torch.floor(yc)
    fx = (xc - x0).to(planes.dtype)
    fy = (yc - y0).to(planes.dtype)
    ix0 = x0.long()
    iy0 = y0.long()
    ix1 = torch.clamp(ix0 + 1, max=w - 1)
    iy1 = torch.clamp(iy0 + 1, max=h - 1)
    flat = planes.reshape(planes.shape[0], -1)

    def at(iy, ix):
        return flat[:, (iy * w + ix).reshape(-1)].reshape((planes.shape[0],) + tuple(x.shape))
    top = (1 - fx) * at(iy0, ix0) + fx * at(iy0, ix1)
    bot = (1 - fx) * at(iy1, ix0) + fx * at(iy1, ix1)
    return (1 - fy) * top + fy * bot


class Unfolding:
    """The unfolded-profile samples of one vortex geometry (centre, r_max), kept on a device so that
    many fields of that geometry are scored without rebuilding them."""

    def __init__(self, cx: float, cy: float, r_max: float, device=None):
        x, y, s = unfolding_grid(cx, cy, r_max)
        self.x = torch.as_tensor(x, device=device, dtype=torch.float64)
        self.y = torch.as_tensor(y, device=device, dtype=torch.float64)
        self.radius = np.abs(s[0])            # the same radii at every angle

    def theory(self, vortex, dtype=torch.float64) -> torch.Tensor:
        """R_th: exact magnitude at each sample radius (independent of the angle) [n_r]."""
        return torch.as_tensor(vortex.magnitude_profile(self.radius), device=self.x.device, dtype=dtype)

    def psi(self, flows: torch.Tensor, r_th: torch.Tensor) -> torch.Tensor:
        """Psi for flows [B, 2, H, W] against per-field theory profiles r_th [B, n_r] (or [n_r])."""
        mag = torch.sqrt(flows[:, 0] ** 2 + flows[:, 1] ** 2)
        r_ofv = _bilinear_many(mag, self.x, self.y)
        th = r_th if r_th.dim() == 2 else r_th[None]
        return torch.mean(torch.abs(r_ofv - th[:, None, :].to(r_ofv.dtype)), dim=(1, 2))


def default_r_max(radius: float, h: int, w: int) -> float:
    return min(2.0 * radius, 0.45 * min(h, w))


def psi(flows: torch.Tensor, vortex, r_max: float = None) -> torch.Tensor:
    """Psi of Eq. (psi_metric) for flows [B, 2, H, W] of one Rankine vortex (synth.Rankine)."""
    _, _, h, w = flows.shape
    if r_max is None:
        r_max = default_r_max(vortex.R, h, w)
    u = Unfolding(vortex.cx, vortex.cy, r_max, flows.device)
    return u.psi(flows, u.theory(vortex, flows.dtype))


def mean_endpoint_error(flows: torch.Tensor, gt: torch.Tensor, border: int) -> torch.Tensor:
    """<Err> over the interior (a band of `border` pixels excluded) for flows [B, 2, H, W] against gt
    [2, H, W] (shared) or [B, 2, H, W]."""
    d = flows - (gt if gt.dim() == 4 else gt[None])
    e = torch.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    if border > 0:
        e = e[:, border:-border, border:-border]
    return e.mean(dim=(1, 2))


def rankine_grid() -> Dict[str, Tuple]:
    """The synthetic-image parameters of the paper's Rankine study (its table of image parameters):
    maximum displacement [px], particles per 16 x 16 interrogation window, core radius [px]."""
    return {"dmax": (8, 16, 24, 32), "part_per_iw": (5, 10, 15), "radius": (12, 25, 50, 75, 100, 150)}


def ofv_grid() -> Dict[str, Tuple]:
    """The estimator parameters of the paper's study (its table of OFV parameter ranges)."""
    return {"kernel_radius": (2, 3, 4, 5, 6, 7), "psl": (2, 3, 4), "iterations": (1, 2, 3, 4),
            "norm_radius": (1, 2, 3, 4)}
