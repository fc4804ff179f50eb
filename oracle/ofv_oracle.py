"""FP64 CPU oracle of the dense optical-flow estimator (test infrastructure).

This module is test infrastructure, not part of the product: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the HIP library.

What it computes is the estimator of the paper's section "Live-Optical Flow
Velocimetry": the symmetric sum-of-squared-differences objective of
Eq. (of_symmetric) over a square window of radius KR around each pixel,
minimised by Gauss-Newton iterations at every level of a Burt-Adelson
Gaussian pyramid, coarse to fine, after a local intensity normalisation
(the six-step pipeline listed in that section).  The method is an iteration,
so the oracle follows its steps in the paper's order, in plain float64 torch
tensor operations (index gathers, arithmetic, floor, clamp, sqrt) with no
blocking or fusion, so that each step can be checked against the text by eye.

Where the paper is silent the following readings are taken (each one is
restated where it is used):

 R1  num_levels is the total number of pyramid levels, PSL + 1.
 R2  REDUCE uses the binomial Burt-Adelson kernel [1, 4, 6, 4, 1] / 16 (a = 3/8),
     replicate border, coarse pixel x sits on fine pixel 2x, coarse size
     ceil(W / 2).
 R3  Normalisation is a local z-score over the (2 NR + 1)^2 window truncated
     to the image: N = (I - mu) / sqrt(sigma^2 + eps) with a two-pass
     variance; NR = 0 means no normalisation.  Integer frames are first
     scaled to [0, 1] by 1 / (2^B - 1).
 R4  The window N(m) is square, unweighted and truncated to the image.
 R5  Gauss-Newton step (Jacobi over pixels): the residual at k is linearised
     about the current flow V(k) there, giving per-pixel rows
     G(k) . V = b(k) with b = G . V(k) - T, solved in the least-squares
     sense over N(m) with Levenberg damping towards V(m):
     (A + lam I) V'(m) = c + lam V(m), lam = reg_rel * trace(A) + reg_abs.
 R6  G is the 3-tap central difference of the warped mean image
     S = (W0 + W1) / 2 with clamped indices; T = W1 - W0.
 R7  Warps are bilinear with sample coordinates clamped to the image.
 R8  Up-sampling is V_fine(X, Y) = 2 * bilinear(V_coarse, X / 2, Y / 2).
 R9  The same IT at every level; V = 0 at the coarsest level, or the
     optional initial field restricted by REDUCE / 2 per level.
 R24 The forward-additive estimator the paper contrasts its symmetric
     objective with (estimator="forward_additive"): the residual
     I1(k + V) - I0(k) is linearised about V(k) with G the central-difference
     gradient of the warped second image, so the step keeps the same normal
     equations with S = W1 = P1(k + V), T = W1 - P0(k); V is then anchored
     at the pixels of frame 0 instead of the midpoint.
 R25 The increment form of the update (update="increment"), the alternative
     to R5: every residual of the window N(m) is linearised about the
     window's own V(m), so G(k) . dV = -T(k) with dV = V - V(m), and
     (A + lam I) dV = sum G (-T), V'(m) = V(m) + dV.  It coincides with R5
     where V is uniform over the window and at V = 0; with the warps of R24
     it is the classic forward-additive Lucas-Kanade step per window.

Besides the method itself, compute_flow can round every image plane (the
normalised frames and each REDUCE output) to a storage type, leaving all
arithmetic in float64.  That is not part of the paper: it gives the error
that storing the planes in float32 / float16 / bfloat16 causes by itself,
the floor against which a reduced-precision implementation is judged.  For
the same purpose it can run every step in float32 arithmetic instead
(arith="f32"): on inputs where the iteration amplifies rounding (windows
whose normal matrix is nearly singular) that is the floor of any float32
implementation.  Both options are diagnostics; the reference is float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

DT = torch.float64


def _t(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(DT) if x.dtype != DT else x
    return torch.as_tensor(np.asarray(x), dtype=DT)


# ---------------------------------------------------------------------------
# Step 1: local intensity normalisation (pipeline step 1; reading R3)
# ---------------------------------------------------------------------------

def intensity(frame, bit_depth: int) -> torch.Tensor:
    """Integer frames scaled to [0, 1] by 1 / (2^B - 1); float frames as given (R3)."""
    if isinstance(frame, np.ndarray) and frame.dtype.kind in "ui":
        return torch.as_tensor(frame.astype(np.float64)) / float(2 ** bit_depth - 1)
    if isinstance(frame, torch.Tensor) and not frame.is_floating_point():
        return frame.to(DT) / float(2 ** bit_depth - 1)
    return _t(frame)


def _shift(x: torch.Tensor, dy: int, dx: int, fill: float = 0.0) -> torch.Tensor:
    """out[y, x] = x[y + dy, x + dx] where inside the image, ``fill`` elsewhere."""
    h, w = x.shape
    out = torch.full_like(x, fill)
    ys0, ys1 = max(0, -dy), min(h, h - dy)
    xs0, xs1 = max(0, -dx), min(w, w - dx)
    if ys0 < ys1 and xs0 < xs1:
        out[ys0:ys1, xs0:xs1] = x[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return out


def window_sum(x: torch.Tensor, radius: int) -> torch.Tensor:
    """Sum over the square window {|dx|, |dy| <= radius} intersected with the image.

    Written as the double sum over window offsets (rows of offsets outer,
    columns inner); pixels outside the image contribute nothing (reading R4).
    """
    out = torch.zeros_like(x)
    for dy in range(-radius, radius + 1):
        row = torch.zeros_like(x)
        for dx in range(-radius, radius + 1):
            row = row + _shift(x, dy, dx)
        out = out + row
    return out


def normalize(i_img: torch.Tensor, nr: int, eps: float) -> torch.Tensor:
    """Pixel-centred local z-score over the truncated (2 NR + 1)^2 window (step 1, R3).

    mu_k = mean of I over the window, sigma_k^2 = mean of (I_j - mu_k)^2 over
    the same window (second pass), N = (I - mu) / sqrt(sigma^2 + eps).
    """
    if nr <= 0:
        return i_img
    ones = torch.ones_like(i_img)
    count = window_sum(ones, nr)
    mu = window_sum(i_img, nr) / count
    var = torch.zeros_like(i_img)
    for dy in range(-nr, nr + 1):
        for dx in range(-nr, nr + 1):
            valid = _shift(ones, dy, dx)
            var = var + valid * (_shift(i_img, dy, dx) - mu) ** 2
    var = var / count
    return (i_img - mu) / torch.sqrt(var + eps)


# ---------------------------------------------------------------------------
# Step 2: Burt-Adelson Gaussian pyramid (pipeline step 2; reading R2)
# ---------------------------------------------------------------------------

BINOMIAL5 = (1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16)


def reduce(p: torch.Tensor) -> torch.Tensor:
    """One REDUCE step: P'(x, y) = sum_{i,j=-2..2} w_i w_j P(cx(2x+i), cy(2y+j)).

    w = [1, 4, 6, 4, 1] / 16, indices clamped into the image, output size
    ceil(H / 2) x ceil(W / 2) (reading R2).
    """
    h, w = p.shape
    hn, wn = (h + 1) // 2, (w + 1) // 2
    ys = torch.arange(hn) * 2
    xs = torch.arange(wn) * 2
    out = torch.zeros((hn, wn), dtype=p.dtype)
    for j in range(-2, 3):
        yy = torch.clamp(ys + j, 0, h - 1)
        for i in range(-2, 3):
            xx = torch.clamp(xs + i, 0, w - 1)
            out = out + BINOMIAL5[j + 2] * BINOMIAL5[i + 2] * p[yy][:, xx]
    return out


_PLANE_TYPES = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def round_plane(p: torch.Tensor, plane_round: Optional[str]) -> torch.Tensor:
    """p rounded to nearest in the storage type (ties to even), back in p's own type."""
    if plane_round is None:
        return p
    return p.to(_PLANE_TYPES[plane_round]).to(p.dtype)


def pyramid(p0: torch.Tensor, levels: int, plane_round: Optional[str] = None) -> List[torch.Tensor]:
    """Levels 0..levels-1; with plane_round each REDUCE reads the rounded finer level."""
    out = [round_plane(p0, plane_round)]
    for _ in range(levels - 1):
        out.append(round_plane(reduce(out[-1]), plane_round))
    return out


# ---------------------------------------------------------------------------
# Step 3: per-pixel symmetric Gauss-Newton at the kernel scale
#         (pipeline steps 3 and 5; Eq. of_symmetric; readings R4-R7)
# ---------------------------------------------------------------------------

def bilinear(p: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Bilinear sample of p at (x, y) with coordinates clamped to the image (R7)."""
    h, w = p.shape
    xc = torch.clamp(x, 0.0, float(w - 1))
    yc = torch.clamp(y, 0.0, float(h - 1))
    x0 = torch.floor(xc)
    y0 = torch.floor(yc)
    fx = xc - x0
    fy = yc - y0
    ix0 = x0.long()
    iy0 = y0.long()
    ix1 = torch.clamp(ix0 + 1, max=w - 1)
    iy1 = torch.clamp(iy0 + 1, max=h - 1)
    p00 = p[iy0, ix0]
    p01 = p[iy0, ix1]
    p10 = p[iy1, ix0]
    p11 = p[iy1, ix1]
    return (1 - fy) * ((1 - fx) * p00 + fx * p01) + fy * ((1 - fx) * p10 + fx * p11)


def central_gradient(s: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """3-tap central differences with clamped indices (R6)."""
    h, w = s.shape
    xi = torch.arange(w)
    yi = torch.arange(h)
    gx = 0.5 * (s[:, torch.clamp(xi + 1, max=w - 1)] - s[:, torch.clamp(xi - 1, min=0)])
    gy = 0.5 * (s[torch.clamp(yi + 1, max=h - 1), :] - s[torch.clamp(yi - 1, min=0), :])
    return gx, gy


@dataclass
class IterationTerms:
    """Intermediate fields of one Gauss-Newton iteration (for stage-level checks)."""
    s: torch.Tensor
    t: torch.Tensor
    gx: torch.Tensor
    gy: torch.Tensor
    b: torch.Tensor
    sums: Dict[str, torch.Tensor] = field(default_factory=dict)


def warp_terms(p0: torch.Tensor, p1: torch.Tensor, u: torch.Tensor, v: torch.Tensor):
    """Midpoint warps of Eq. (of_symmetric): W0 = P0(k - V/2), W1 = P1(k + V/2).

    Returns S = (W0 + W1) / 2 and T = W1 - W0 at every pixel k (R6, R7).
    """
    h, w = p0.shape
    yy, xx = torch.meshgrid(torch.arange(h, dtype=p0.dtype), torch.arange(w, dtype=p0.dtype), indexing="ij")
    w0 = bilinear(p0, xx - 0.5 * u, yy - 0.5 * v)
    w1 = bilinear(p1, xx + 0.5 * u, yy + 0.5 * v)
    return 0.5 * (w0 + w1), w1 - w0


def warp_terms_forward(p0: torch.Tensor, p1: torch.Tensor, u: torch.Tensor, v: torch.Tensor):
    """Forward-additive warps (R24): W1 = P1(k + V); S = W1 and T = W1 - P0(k)."""
    h, w = p0.shape
    yy, xx = torch.meshgrid(torch.arange(h, dtype=p0.dtype), torch.arange(w, dtype=p0.dtype), indexing="ij")
    w1 = bilinear(p1, xx + u, yy + v)
    return w1, w1 - p0


def increment_step(a, d, sxy, det, sxb, syb, u, v):
    """R25: the damped step dV = (A + lam I)^-1 c by Cramer's rule (a, d the damped diagonal,
    det its determinant, c = (sxb, syb) the sums of G (-T)), added to the current V(m)."""
    return u + (d * sxb - sxy * syb) / det, v + (a * syb - sxy * sxb) / det


def gn_iteration(p0: torch.Tensor, p1: torch.Tensor, u: torch.Tensor, v: torch.Tensor,
                 kr: int, reg_rel: float, reg_abs: float, terms: Optional[list] = None,
                 estimator: str = "symmetric", update: str = "consistent"):
    """One Jacobi Gauss-Newton update of the flow at every pixel (R5).

    At each pixel k the residual I0(k - V/2) - I1(k + V/2) of Eq. (of_symmetric)
    is linearised about V(k): it equals -(T + G . (V - V(k))) to first order,
    with G = grad S.  Requiring V constant on N(m) and minimising the sum of
    squares gives the normal equations A V = c with
        A = sum_{k in N(m)} G G^T,   c = sum_{k in N(m)} G b,   b = G . V(k) - T.
    With damping lam = reg_rel (Sxx + Syy) + reg_abs towards the current V(m),
    (A + lam I) V'(m) = c + lam V(m) is solved by Cramer's rule.
    estimator="forward_additive" takes the warps of R24 instead.
    update="increment" (R25): b = -T, (A + lam I) dV = c, V'(m) = V(m) + dV.
    """
    if estimator == "symmetric":
        s, t = warp_terms(p0, p1, u, v)
    elif estimator == "forward_additive":
        s, t = warp_terms_forward(p0, p1, u, v)
    else:
        raise ValueError(f"unknown estimator {estimator!r}")
    gx, gy = central_gradient(s)
    if update == "consistent":
        b = gx * u + gy * v - t
    elif update == "increment":
        b = -t
    else:
        raise ValueError(f"unknown update {update!r}")
    sxx = window_sum(gx * gx, kr)
    sxy = window_sum(gx * gy, kr)
    syy = window_sum(gy * gy, kr)
    sxb = window_sum(gx * b, kr)
    syb = window_sum(gy * b, kr)
    lam = reg_rel * (sxx + syy) + reg_abs
    a = sxx + lam
    d = syy + lam
    det = a * d - sxy * sxy
    if update == "consistent":
        r1 = sxb + lam * u
        r2 = syb + lam * v
        un = (d * r1 - sxy * r2) / det
        vn = (a * r2 - sxy * r1) / det
    else:
        un, vn = increment_step(a, d, sxy, det, sxb, syb, u, v)
    if terms is not None:
        terms.append(IterationTerms(s, t, gx, gy, b, {"sxx": sxx, "sxy": sxy, "syy": syy,
                                                       "sxb": sxb, "syb": syb}))
    return un, vn


# ---------------------------------------------------------------------------
# Step 4: up-sampling and projection to the next finer level (pipeline step 4; R8)
# ---------------------------------------------------------------------------

def upsample(uc: torch.Tensor, vc: torch.Tensor, h: int, w: int):
    """V_fine(X, Y) = 2 * bilinear(V_coarse, X / 2, Y / 2) on an h x w grid (R8)."""
    yy, xx = torch.meshgrid(torch.arange(h, dtype=uc.dtype), torch.arange(w, dtype=uc.dtype), indexing="ij")
    return 2.0 * bilinear(uc, 0.5 * xx, 0.5 * yy), 2.0 * bilinear(vc, 0.5 * xx, 0.5 * yy)


def restrict_flow(u: torch.Tensor, v: torch.Tensor):
    """Initial field at the next coarser level: REDUCE(V) / 2 per component (R9)."""
    return 0.5 * reduce(u), 0.5 * reduce(v)


# ---------------------------------------------------------------------------
# Whole pipeline (steps 1-6)
# ---------------------------------------------------------------------------

DEFAULTS = {"norm_eps": 1e-4, "reg_rel": 1e-3, "reg_abs": 1e-9}


@dataclass
class Trace:
    """Optional record of every intermediate, for stage-level comparisons."""
    levels0: List[torch.Tensor] = field(default_factory=list)
    levels1: List[torch.Tensor] = field(default_factory=list)
    flow_in: Dict[int, Tuple[torch.Tensor, torch.Tensor]] = field(default_factory=dict)
    iterates: Dict[Tuple[int, int], Tuple[torch.Tensor, torch.Tensor]] = field(default_factory=dict)


def compute_flow(frame0, frame1, params: Dict, bit_depth0: int = 8, bit_depth1: Optional[int] = None,
                 flow_init=None, trace: Optional[Trace] = None, plane_round: Optional[str] = None,
                 arith: Optional[str] = None):
    """Dense displacement field (u, v) in px/frame at full resolution.

    params: num_levels (PSL + 1), kernel_radius (KR), iterations (IT),
    norm_radius (NR), and optionally norm_eps, reg_rel, reg_abs,
    estimator ("symmetric", the paper's, or "forward_additive", R24) and
    update ("consistent", R5, or "increment", R25).
    Returns a float64 tensor [2, H, W]; u along +x (columns), v along +y
    (rows), mapping frame0 to frame1, defined at the midpoint.
    plane_round ("f32", "f16", "bf16" or None) rounds every image plane to
    that storage type; arith="f32" runs every step in float32 (both not part
    of the method; see the module docstring).
    """
    if bit_depth1 is None:
        bit_depth1 = bit_depth0
    p = dict(DEFAULTS)
    p.update(params)
    levels = int(p["num_levels"])
    kr = int(p["kernel_radius"])
    it = int(p["iterations"])
    nr = int(p["norm_radius"])
    # step 1: normalisation of each frame, independently
    dt = torch.float32 if arith == "f32" else DT
    n0 = normalize(intensity(frame0, bit_depth0).to(dt), nr, p["norm_eps"])
    n1 = normalize(intensity(frame1, bit_depth1).to(dt), nr, p["norm_eps"])
    # step 2: pyramids
    pyr0 = pyramid(n0, levels, plane_round)
    pyr1 = pyramid(n1, levels, plane_round)
    if trace is not None:
        trace.levels0, trace.levels1 = pyr0, pyr1
    # initial flow at the coarsest level
    hc, wc = pyr0[-1].shape
    if flow_init is None:
        u = torch.zeros((hc, wc), dtype=dt)
        v = torch.zeros((hc, wc), dtype=dt)
    else:
        fi = _t(flow_init).to(dt)
        u, v = fi[0], fi[1]
        for _ in range(levels - 1):
            u, v = restrict_flow(u, v)
    # steps 3-5: coarse to fine
    for lev in range(levels - 1, -1, -1):
        if lev < levels - 1:
            h, w = pyr0[lev].shape
            u, v = upsample(u, v, h, w)
        if trace is not None:
            trace.flow_in[lev] = (u, v)
        for k in range(it):
            u, v = gn_iteration(pyr0[lev], pyr1[lev], u, v, kr, p["reg_rel"], p["reg_abs"],
                                estimator=p.get("estimator", "symmetric"), update=p.get("update", "consistent"))
            if trace is not None:
                trace.iterates[(lev, k)] = (u, v)
    # step 6: full-resolution field
    return torch.stack([u, v]).to(DT)


def endpoint_error(flow, gt) -> torch.Tensor:
    """Err(x, y) = sqrt(du^2 + dv^2), Eq. (absolute_error)."""
    f = _t(flow)
    g = _t(gt)
    return torch.sqrt((f[0] - g[0]) ** 2 + (f[1] - g[1]) ** 2)
