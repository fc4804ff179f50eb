"""Brute-force reference for tiny images: scalar Python loops and numpy.linalg.

Structurally independent of the oracle: every quantity is computed pixel by
pixel with scalar arithmetic, and each Gauss-Newton step assembles the
per-window least-squares problem explicitly (one row per pixel of the
window) and hands it to numpy.linalg.solve.  Used only on inputs of a few
dozen pixels.
"""
from __future__ import annotations

import math
import statistics
from typing import List, Optional

import numpy as np

W5 = [1.0, 4.0, 6.0, 4.0, 1.0]


def bf_normalize(img: np.ndarray, nr: int, eps: float) -> np.ndarray:
    h, w = img.shape
    if nr == 0:
        return img.astype(np.float64).copy()
    out = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            vals = [float(img[j, i]) for j in range(max(0, y - nr), min(h, y + nr + 1))
                    for i in range(max(0, x - nr), min(w, x + nr + 1))]
            mu = statistics.fmean(vals)
            var = statistics.pvariance(vals, mu)
            out[y, x] = (float(img[y, x]) - mu) / math.sqrt(var + eps)
    return out


def bf_reduce(p: np.ndarray) -> np.ndarray:
    h, w = p.shape
    hn, wn = (h + 1) // 2, (w + 1) // 2
    out = np.zeros((hn, wn))
    for y in range(hn):
        for x in range(wn):
            acc = 0.0
            for j in range(5):
                for i in range(5):
                    yy = min(max(2 * y + j - 2, 0), h - 1)
                    xx = min(max(2 * x + i - 2, 0), w - 1)
                    acc += W5[j] * W5[i] * float(p[yy, xx])
            out[y, x] = acc / 256.0
    return out


def bf_bilinear(p: np.ndarray, x: float, y: float) -> float:
    h, w = p.shape
    x = min(max(x, 0.0), w - 1.0)
    y = min(max(y, 0.0), h - 1.0)
    x0, y0 = int(math.floor(x)), int(math.floor(y))
    x1, y1 = min(x0 + 1, w - 1), min(y0 + 1, h - 1)
    ax, ay = x - x0, y - y0
    top = float(p[y0, x0]) + ax * (float(p[y0, x1]) - float(p[y0, x0]))
    bot = float(p[y1, x0]) + ax * (float(p[y1, x1]) - float(p[y1, x0]))
    return top + ay * (bot - top)


def bf_gn_iteration(p0: np.ndarray, p1: np.ndarray, u: np.ndarray, v: np.ndarray, kr: int,
                    reg_rel: float, reg_abs: float, forward_additive: bool = False, increment: bool = False):
    """One Jacobi step: per-window least squares with Levenberg damping rows.

    For every m, the linear model of the residual at each k in the window is
    G(k) . V ~= G(k) . V(k) - T(k); damping adds sqrt(lam) * (V - V(m)) = 0
    rows.  The normal equations of that stacked system are solved with
    numpy.linalg.solve.  increment: the unknown is the step D = V - V(m) and
    the model at every k of the window is G(k) . D ~= -T(k), damping rows
    sqrt(lam) * D = 0; the result is V(m) + D.
    """
    h, w = p0.shape
    s = np.zeros((h, w))
    t = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            if forward_additive:   # I1(k + V) - I0(k), gradient of the warped second image
                w0 = p0[y, x]
                w1 = bf_bilinear(p1, x + u[y, x], y + v[y, x])
                s[y, x] = w1
            else:
                w0 = bf_bilinear(p0, x - u[y, x] / 2.0, y - v[y, x] / 2.0)
                w1 = bf_bilinear(p1, x + u[y, x] / 2.0, y + v[y, x] / 2.0)
                s[y, x] = (w0 + w1) / 2.0
            t[y, x] = w1 - w0
    g = np.zeros((h, w, 2))
    for y in range(h):
        for x in range(w):
            g[y, x, 0] = (s[y, min(x + 1, w - 1)] - s[y, max(x - 1, 0)]) / 2.0
            g[y, x, 1] = (s[min(y + 1, h - 1), x] - s[max(y - 1, 0), x]) / 2.0
    un = np.zeros((h, w))
    vn = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            rows: List[np.ndarray] = []
            rhs: List[float] = []
            for yy in range(max(0, y - kr), min(h, y + kr + 1)):
                for xx in range(max(0, x - kr), min(w, x + kr + 1)):
                    gk = g[yy, xx]
                    rows.append(gk)
                    if increment:
                        rhs.append(float(-t[yy, xx]))
                    else:
                        rhs.append(float(gk[0] * u[yy, xx] + gk[1] * v[yy, xx] - t[yy, xx]))
            a = np.array(rows)
            bvec = np.array(rhs)
            lam = reg_rel * float(np.sum(a * a)) + reg_abs
            if increment:
                stacked = np.vstack([a, math.sqrt(lam) * np.eye(2)])
                target = np.concatenate([bvec, np.zeros(2)])
                step = np.linalg.solve(stacked.T @ stacked, stacked.T @ target)
                un[y, x], vn[y, x] = u[y, x] + step[0], v[y, x] + step[1]
                continue
            normal = a.T @ a + lam * np.eye(2)
            rhs_n = a.T @ bvec + lam * np.array([u[y, x], v[y, x]])
            sol = np.linalg.solve(normal, rhs_n)
            un[y, x], vn[y, x] = sol
    return un, vn


def bf_upsample(uc: np.ndarray, h: int, w: int) -> np.ndarray:
    out = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            out[y, x] = 2.0 * bf_bilinear(uc, x / 2.0, y / 2.0)
    return out


def bf_compute_flow(i0: np.ndarray, i1: np.ndarray, levels: int, kr: int, it: int, nr: int,
                    eps: float, reg_rel: float, reg_abs: float,
                    flow_init: Optional[np.ndarray] = None, forward_additive: bool = False,
                    increment: bool = False) -> np.ndarray:
    """The whole pipeline on float intensity images (already scaled to [0, 1])."""
    n0 = bf_normalize(i0, nr, eps)
    n1 = bf_normalize(i1, nr, eps)
    pyr0, pyr1 = [n0], [n1]
    for _ in range(levels - 1):
        pyr0.append(bf_reduce(pyr0[-1]))
        pyr1.append(bf_reduce(pyr1[-1]))
    hc, wc = pyr0[-1].shape
    if flow_init is None:
        u = np.zeros((hc, wc))
        v = np.zeros((hc, wc))
    else:
        u, v = flow_init[0].astype(np.float64), flow_init[1].astype(np.float64)
        for _ in range(levels - 1):
            u, v = bf_reduce(u) / 2.0, bf_reduce(v) / 2.0
    for lev in range(levels - 1, -1, -1):
        h, w = pyr0[lev].shape
        if lev < levels - 1:
            u, v = bf_upsample(u, h, w), bf_upsample(v, h, w)
        for _ in range(it):
            u, v = bf_gn_iteration(pyr0[lev], pyr1[lev], u, v, kr, reg_rel, reg_abs, forward_additive, increment)
    return np.stack([u, v])
