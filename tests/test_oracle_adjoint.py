"""The oracle's autograd (the reference adjoint) against central finite differences (CPU).

Loss L = sum |V - V_gt|^2 on a 32 x 32 float-frame crop.  The estimator is
piecewise smooth: bilinear weights have kinks where a sample crosses an
integer coordinate, so a few finite differences straddle a kink; their count
is reported and must stay a small minority.
"""
import numpy as np
import torch

import oracle
import synth

H = 1e-3


def _setup():
    pair = synth.make_pair(32, 32, synth.Rankine(15.5, 16.0, 8.0, 1.5), fwhm=2.5, ppp=0.1, seed=77, bit_depth=0,
                           noise=2.0 / 255.0)
    prm = {"num_levels": 2, "kernel_radius": 2, "iterations": 2, "norm_radius": 1}
    init = pair.gt + np.random.default_rng(5).normal(0, 0.2, pair.gt.shape)
    return pair, prm, init


def _loss(f0, f1, init, prm, gt):
    v = oracle.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init)
    return torch.sum((v - gt) ** 2)


def test_oracle_autograd_matches_central_differences():
    pair, prm, init = _setup()
    gt = torch.as_tensor(pair.gt)
    x0 = torch.as_tensor(pair.frame0.astype(np.float64)).requires_grad_(True)
    x1 = torch.as_tensor(pair.frame1.astype(np.float64)).requires_grad_(True)
    xi = torch.as_tensor(init).requires_grad_(True)
    loss = _loss(x0, x1, xi, prm, gt)
    g0, g1, gi = torch.autograd.grad(loss, [x0, x1, xi])
    rng = np.random.default_rng(9)
    checked = kinks = 0
    for name, base, grad in (("frame0", x0, g0), ("frame1", x1, g1), ("flow_init", xi, gi)):
        flat = base.detach().clone().reshape(-1)
        gflat = grad.reshape(-1)
        scale = float(gflat.abs().max())
        for idx in rng.choice(flat.numel(), 16, replace=False):
            def at(delta):
                z = flat.clone()
                z[idx] += delta
                z = z.reshape(base.shape)
                args = {"frame0": (z, x1.detach(), xi.detach()), "frame1": (x0.detach(), z, xi.detach()),
                        "flow_init": (x0.detach(), x1.detach(), z)}[name]
                return float(_loss(*args, prm, gt))
            fd = (at(H) - at(-H)) / (2 * H)
            ad = float(gflat[idx])
            checked += 1
            if abs(fd - ad) > 1e-4 * max(abs(ad), 1e-2 * scale):
                kinks += 1
    print(f"finite differences: {checked} checked, {kinks} straddle a kink")
    assert kinks <= checked // 8
