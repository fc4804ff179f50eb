"""The oracle's autograd (the reference adjoint) against central finite differences (CPU).

Loss L = sum |V - V_gt|^2 on a 32 x 32 float-frame crop, central finite
differences with h = 1e-3 and one Richardson step (the differences at h and
h/2 combined to cancel the h^2 term): the local z-score is curved enough at
the scale of 1e-3 intensity units that plain central differences miss the
1e-5 bar by their truncation error alone (their error is reported beside).
The estimator is piecewise smooth: its only kinks are the floor and the
clamp inside bilinear interpolation (warps and up-sampling).  A sample
straddles a kink when its perturbations change any floor index or clamp
outcome of the forward pass; such samples are detected by recording those
outcomes (not guessed from the size of the error), counted and reported,
and every other sample must agree with autograd to 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import ofv_oracle as O

H = 1e-3
REL = 1e-5


def _setup(seed=77):
    pair = synth.make_pair(32, 32, synth.Rankine(15.5, 16.0, 8.0, 1.5), fwhm=2.5, ppp=0.1, seed=seed, bit_depth=0,
                           noise=2.0 / 255.0)
    prm = {"num_levels": 2, "kernel_radius": 2, "iterations": 2, "norm_radius": 1}
    init = pair.gt + np.random.default_rng(5).normal(0, 0.2, pair.gt.shape)
    return pair, prm, init


def _loss(f0, f1, init, prm, gt):
    v = oracle.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init)
    return torch.sum((v - gt) ** 2)


class _KinkRecorder:
    """Wraps the oracle's bilinear interpolation and records, for every call of a forward pass,
    the floor of the clamped coordinates and which coordinates were clamped."""

    def __init__(self, monkeypatch):
        self.orig = O.bilinear
        self.log = None
        monkeypatch.setattr(O, "bilinear", self._bilinear)

    def _bilinear(self, p, x, y):
        if self.log is not None:
            h, w = p.shape
            xd, yd = x.detach(), y.detach()
            self.log.append(torch.stack([torch.floor(torch.clamp(xd, 0.0, float(w - 1))),
                                         torch.floor(torch.clamp(yd, 0.0, float(h - 1))),
                                         (xd < 0).double(), (xd > w - 1).double(),
                                         (yd < 0).double(), (yd > h - 1).double()]))
        return self.orig(p, x, y)

    def run(self, fn):
        self.log = []
        out = fn()
        log, self.log = self.log, None
        return out, log


def _straddles(log_a, log_b):
    return len(log_a) != len(log_b) or any(not torch.equal(a, b) for a, b in zip(log_a, log_b))


def _fd_check(monkeypatch, pair, prm, init, n_per_input, seed):
    rec = _KinkRecorder(monkeypatch)
    gt = torch.as_tensor(pair.gt)
    x0 = torch.as_tensor(pair.frame0.astype(np.float64)).requires_grad_(True)
    x1 = torch.as_tensor(pair.frame1.astype(np.float64)).requires_grad_(True)
    xi = torch.as_tensor(init).requires_grad_(True)
    loss = _loss(x0, x1, xi, prm, gt)
    g0, g1, gi = torch.autograd.grad(loss, [x0, x1, xi])
    rng = np.random.default_rng(seed)
    rows = []
    for name, base, grad in (("frame0", x0, g0), ("frame1", x1, g1), ("flow_init", xi, gi)):
        flat = base.detach().clone().reshape(-1)
        gflat = grad.reshape(-1)
        scale = float(gflat.abs().max())
        for idx in rng.choice(flat.numel(), n_per_input, replace=False):
            def at(delta):
                z = flat.clone()
                z[idx] += delta
                z = z.reshape(base.shape)
                args = {"frame0": (z, x1.detach(), xi.detach()), "frame1": (x0.detach(), z, xi.detach()),
                        "flow_init": (x0.detach(), x1.detach(), z)}[name]
                return rec.run(lambda: float(_loss(*args, prm, gt)))
            (lp, log_p), (lm, log_m) = at(H), at(-H)
            (lp2, log_p2), (lm2, log_m2) = at(H / 2), at(-H / 2)
            fd_h = (lp - lm) / (2 * H)
            fd_h2 = (lp2 - lm2) / H
            fd = (4.0 * fd_h2 - fd_h) / 3.0
            ad = float(gflat[idx])
            den = max(abs(ad), 1e-3 * scale)
            kink = _straddles(log_p, log_m) or _straddles(log_p2, log_m2) or _straddles(log_p, log_p2)
            rows.append((name, int(idx), ad, fd, abs(fd - ad) / den, kink, abs(fd_h - ad) / den))
    return rows


def test_oracle_autograd_matches_central_differences(monkeypatch):
    pair, prm, init = _setup()
    rows = _fd_check(monkeypatch, pair, prm, init, 24, seed=9)
    kinks = [r for r in rows if r[5]]
    smooth = [r for r in rows if not r[5]]
    worst = max(r[4] for r in smooth)
    worst_plain = max(r[6] for r in smooth)
    print(f"finite differences: {len(rows)} checked, {len(kinks)} straddle a kink (excluded); "
          f"worst relative error of the rest {worst:.2e} (plain central differences {worst_plain:.2e})")
    assert len(smooth) >= 3 * len(rows) // 4
    bad = [r for r in smooth if r[4] > REL]
    assert not bad, bad[:5]


def test_kink_detection_sees_a_planted_kink(monkeypatch):
    """A perturbation that moves a warp sample across an integer coordinate is reported as a
    kink: the flow_init entry of a pixel whose warped x sits within h of an integer."""
    pair, prm, init = _setup()
    prm1 = dict(prm, num_levels=1, iterations=1)
    # put the warp samples of pixel (16, 16) exactly on integers: u = 2 gives x -/+ 1 there
    init = init.copy()
    init[0, 16, 16] = 2.0
    rec = _KinkRecorder(monkeypatch)
    gt = torch.as_tensor(pair.gt)

    def loss_at(delta):
        z = init.copy()
        z[0, 16, 16] += delta
        return rec.run(lambda: float(_loss(pair.frame0, pair.frame1, z, prm1, gt)))
    (_, lp), (_, lm) = loss_at(H), loss_at(-H)
    assert _straddles(lp, lm)
    (_, lp), (_, lm) = loss_at(0.3 + H), loss_at(0.3 - H)
    assert not _straddles(lp, lm)
