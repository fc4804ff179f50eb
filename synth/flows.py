"""Analytic displacement fields (px/frame) used to advect synthetic particles.

Coordinates: x along columns, y along rows, pixel centres at integers.  Each
field is a callable ``flow(x, y) -> (dx, dy)`` on equal-shape float64 arrays;
fields that are expensive to evaluate point-wise also expose
``grid(h, w)`` returning the [h, w] components directly.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


class Translation:
    """Uniform translation (tx, ty) plus an optional linear shear of du/dy."""

    def __init__(self, tx: float, ty: float, shear: float = 0.0, y_ref: float = 0.0):
        self.tx, self.ty, self.shear, self.y_ref = tx, ty, shear, y_ref

    def __call__(self, x, y):
        dx = self.tx + self.shear * (y - self.y_ref)
        dy = np.full_like(np.asarray(y, dtype=np.float64), self.ty)
        return np.broadcast_to(dx, np.shape(x)).astype(np.float64), dy


class Rankine:
    """Rankine vortex, following the analytic description in the paper's
    "Rankine vortex" subsection (boxed formula): azimuthal displacement
    u_theta(r) = D * (r/R) inside the core and D * (R/r) outside, where D is
    the maximum displacement (Gamma / (2 pi M R) in the paper's notation),
    and particles move by a rotation of angle u_theta / r about the centre.

    The boxed formula gives the new particle position.  The displacement is
    the chord of that rotation; split symmetrically about the midpoint
    position it is 2 sin(phi / 2) * (-(y - cy), x - cx) with phi = u_theta / r
    (positive rotation from +x towards +y).
    """

    def __init__(self, cx: float, cy: float, radius: float, dmax: float):
        self.cx, self.cy, self.R, self.D = cx, cy, radius, dmax

    def __call__(self, x, y):
        rx = np.asarray(x, dtype=np.float64) - self.cx
        ry = np.asarray(y, dtype=np.float64) - self.cy
        r2 = rx * rx + ry * ry
        inside = r2 <= self.R * self.R
        with np.errstate(divide="ignore", invalid="ignore"):
            phi = np.where(inside, self.D / self.R, self.D * self.R / np.where(inside, 1.0, r2))
        s = 2.0 * np.sin(0.5 * phi)
        return -s * ry, s * rx

    def magnitude_profile(self, r):
        """Exact chord magnitude |d| at radius r (used for the radial-profile check)."""
        r = np.asarray(r, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            phi = np.where(r <= self.R, self.D / self.R, self.D * self.R / np.maximum(r, 1e-300) ** 2)
        return 2.0 * r * np.sin(0.5 * phi)


class Turbulence:
    """Divergence-free random-Fourier-mode field with an E(k) ~ k^(-5/3) spectrum.

    Stream function psi = sum_j a_j sin(k_j . x + phi_j(t)), d = (dpsi/dy, -dpsi/dx).
    |k_j| is log-stratified in [2 pi / 1024, 2 pi / 16] px^-1 with random
    directions; the displacement amplitude of mode j is proportional to
    |k_j|^(-1/3), i.e. an energy density ~ k^(-5/3) over log-spaced modes.
    phi_j(t) = phi_j + 2 pi t / T_j with T_j = 64 (k_j / k_min)^(-2/3) frames.
    The field is scaled to the requested RMS displacement over an
    ``ref_h`` x ``ref_w`` grid at t = 0; a draw whose maximum there exceeds
    ``dmax_cap`` is redrawn with the next seed.
    """

    def __init__(self, seed: int, n_modes: int = 256, rms: float = 2.0, dmax_cap: float = 8.0,
                 ref_h: int = 256, ref_w: int = 256, t: float = 0.0,
                 kmin: float = 2 * math.pi / 1024, kmax: float = 2 * math.pi / 16):
        for attempt in range(64):
            rng = np.random.default_rng(seed + 100_003 * attempt)
            j = np.arange(n_modes)
            kmag = kmin * (kmax / kmin) ** ((j + rng.uniform(0, 1, n_modes)) / n_modes)
            th = rng.uniform(0, 2 * math.pi, n_modes)
            self.kx = kmag * np.cos(th)
            self.ky = kmag * np.sin(th)
            self.phase0 = rng.uniform(0, 2 * math.pi, n_modes)
            self.period = 64.0 * (kmag / kmin) ** (-2.0 / 3.0)
            amp_disp = kmag ** (-1.0 / 3.0)
            self.a = amp_disp / kmag
            self.kmag = kmag
            self.t = 0.0
            u, v = self.grid(ref_h, ref_w)
            scale = rms / math.sqrt(float(np.mean(u * u + v * v)))
            self.a = self.a * scale
            if float(np.max(np.hypot(u, v))) * scale <= dmax_cap:
                break
        self.t = t
        self.seed_used = seed + 100_003 * attempt

    def _phase(self):
        return self.phase0 + 2 * math.pi * self.t / self.period

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        flat_x, flat_y = x.ravel(), y.ravel()
        u = np.zeros_like(flat_x)
        v = np.zeros_like(flat_x)
        ph = self._phase()
        for s in range(0, flat_x.size, 65536):
            arg = (flat_x[s:s + 65536, None] * self.kx[None, :] + flat_y[s:s + 65536, None] * self.ky[None, :]
                   + ph[None, :])
            c = np.cos(arg) * self.a[None, :]
            u[s:s + 65536] = c @ self.ky
            v[s:s + 65536] = -(c @ self.kx)
        return u.reshape(x.shape), v.reshape(x.shape)

    def grid(self, h: int, w: int) -> Tuple[np.ndarray, np.ndarray]:
        xs = np.arange(w, dtype=np.float64)
        ys = np.arange(h, dtype=np.float64)
        ph = self._phase()
        cxs, sxs = np.cos(np.outer(self.kx, xs)), np.sin(np.outer(self.kx, xs))          # [n, w]
        ay = np.outer(ys, self.ky) + ph[None, :]                                           # [h, n]
        cy, sy = np.cos(ay) * self.a[None, :], np.sin(ay) * self.a[None, :]
        # cos(kx x + ky y + p) = cos(kx x) cos(ky y + p) - sin(kx x) sin(ky y + p)
        u = (cy * self.ky) @ cxs - (sy * self.ky) @ sxs
        v = -((cy * self.kx) @ cxs - (sy * self.kx) @ sxs)
        return u, v


class CylinderWake:
    """Potential flow past a cylinder plus an alternating Lamb-Oseen vortex street.

    Complex velocity u - i v = U (1 - a^2 / (z - z0)^2) outside the cylinder
    (zero inside); vortices of core radius rc with alternating circulation
    +-Gamma sit at x = x0 + a + (n + t/T) lambda / 2, y = y0 -+ h/2 and drift
    downstream with period T.  The whole field is scaled so that its maximum
    over the image is ``dmax``.
    """

    def __init__(self, h: int, w: int, x0: float = 1024.0, y0: float = 2048.0, a: float = 200.0,
                 rc: float = 100.0, wavelength: float = 1800.0, spacing_ratio: float = 0.28,
                 period: float = 200.0, t: float = 0.0, dmax: float = 10.0):
        self.x0, self.y0, self.a, self.rc = x0, y0, a, rc
        self.lam, self.hs, self.T, self.t = wavelength, spacing_ratio * wavelength, period, t
        self.scale = 1.0
        n_vort = int(math.ceil((w - x0) / (0.5 * wavelength))) + 2
        self.n_vort = n_vort
        u, v = self._raw_grid(min(h, 1024), min(w, 1024), h, w)
        m = float(np.max(np.hypot(u, v)))
        self.scale = dmax / m if m > 0 else 1.0

    def _raw(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        z = (x - self.x0) + 1j * (y - self.y0)
        inside = np.abs(z) < self.a
        zz = np.where(inside, 1.0 + 0j, z)
        wv = 1.0 - (self.a ** 2) / (zz * zz)
        u, v = wv.real.copy(), -wv.imag
        gamma = 2 * math.pi * self.rc * 0.6
        frac = (self.t / self.T) % 1.0
        for n in range(self.n_vort):
            xv = self.x0 + self.a + (n + frac) * 0.5 * self.lam
            yv = self.y0 + (0.5 * self.hs if n % 2 else -0.5 * self.hs)
            g = gamma if n % 2 == 0 else -gamma
            rx, ry = x - xv, y - yv
            r2 = rx * rx + ry * ry + 1e-12
            f = g / (2 * math.pi * r2) * (1.0 - np.exp(-r2 / (self.rc ** 2)))
            u = u - f * ry
            v = v + f * rx
        u = np.where(inside, 0.0, u)
        v = np.where(inside, 0.0, v)
        return u, v

    def _raw_grid(self, hs, ws, h, w):
        ys = np.linspace(0, h - 1, hs)
        xs = np.linspace(0, w - 1, ws)
        gx, gy = np.meshgrid(xs, ys)
        return self._raw(gx, gy)

    def inside(self, x, y):
        return np.hypot(np.asarray(x) - self.x0, np.asarray(y) - self.y0) < self.a

    def __call__(self, x, y):
        u, v = self._raw(x, y)
        return u * self.scale, v * self.scale
