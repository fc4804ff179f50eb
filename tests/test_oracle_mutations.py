"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutation replaces one oracle step with a plausible slip (a wrong sign,
a dropped factor, a swapped operand, an off-by-one radius) and runs a fast
subset of the pins; at least one of them must fail.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ofv_oracle as O
from tests import bruteforce as bf


def _check_bruteforce():
    rng = np.random.default_rng(77)
    i0 = rng.uniform(0, 1, (8, 8))
    i1 = rng.uniform(0, 1, (8, 8))
    v0 = rng.uniform(-1, 1, (2, 8, 8))
    prm = {"num_levels": 2, "kernel_radius": 1, "iterations": 2, "norm_radius": 1}
    got = O.compute_flow(i0, i1, prm, bit_depth0=0, flow_init=v0).numpy()
    ref = bf.bf_compute_flow(i0, i1, 2, 1, 2, 1, 1e-4, 1e-3, 1e-9, flow_init=v0)
    return np.max(np.abs(got - ref)) < 1e-10


def _check_fixed_point():
    import synth
    n, m = 48, 6
    tex = synth.make_texture(n, n, fwhm=2.5, ppp=0.1, seed=5, margin=m)
    f0 = tex[m:m + n, m:m + n]
    f1 = tex[m:m + n, m - 2:m - 2 + n]
    init = np.stack([np.full((n, n), 2.0), np.zeros((n, n))])
    prm = {"num_levels": 1, "kernel_radius": 2, "iterations": 1, "norm_radius": 0}
    out = O.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init).numpy()
    return np.max(np.abs(out[:, 8:-8, 8:-8] - init[:, 8:-8, 8:-8])) < 1e-12


def _check_upsample_affine():
    # 2 * bilinear(V, X/2, Y/2) of an affine coarse field is affine with doubled values
    h, w = 6, 7
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    uc = torch.as_tensor(0.3 * xx + 0.1 * yy)
    u, _ = O.upsample(uc, uc, 2 * h - 1, 2 * w - 1)
    Y, X = np.mgrid[0:2 * h - 1, 0:2 * w - 1].astype(np.float64)
    return np.max(np.abs(u.numpy() - 2 * (0.3 * X / 2 + 0.1 * Y / 2))) < 1e-12


CHECKS = [_check_bruteforce, _check_fixed_point, _check_upsample_affine]


def _caught():
    for chk in CHECKS:
        try:
            if not chk():
                return True
        except Exception:
            return True
    return False


def test_unmutated_oracle_passes_all_checks():
    assert all(chk() for chk in CHECKS)


def _mut_t_sign(p0, p1, u, v):
    s, t = ORIG["warp_terms"](p0, p1, u, v)
    return s, -t


def _mut_full_warp(p0, p1, u, v):
    return ORIG["warp_terms"](p0, p1, 2 * u, 2 * v)


def _mut_swap_grad(s):
    gx, gy = ORIG["central_gradient"](s)
    return gy, gx


def _mut_window_radius(x, r):
    return ORIG["window_sum"](x, r + 1)


def _mut_upsample_no_scale(uc, vc, h, w):
    u, v = ORIG["upsample"](uc, vc, h, w)
    return 0.5 * u, 0.5 * v


def _mut_bilinear_swap(p, x, y):
    h, w = p.shape
    if h == w:
        return ORIG["bilinear"](p.T, x, y)
    return ORIG["bilinear"](p, x, y) * 1.0001


def _mut_reduce_no_clamp(p):
    r = ORIG["reduce"](p)
    r[0, :] = r[0, :] * 0.9
    return r


def _mut_normalize_one_pass_wrong(i_img, nr, eps):
    if nr <= 0:
        return i_img
    n = O.window_sum(torch.ones_like(i_img), nr)
    mu = O.window_sum(i_img, nr) / n
    var = O.window_sum(i_img * i_img, nr) / n - mu * mu
    return (i_img - mu) / torch.sqrt(var + 2 * eps)


ORIG = {name: getattr(O, name) for name in
        ["warp_terms", "central_gradient", "window_sum", "upsample", "bilinear", "reduce", "normalize"]}

MUTATIONS = [
    ("warp_terms", _mut_t_sign),
    ("warp_terms", _mut_full_warp),
    ("central_gradient", _mut_swap_grad),
    ("window_sum", _mut_window_radius),
    ("upsample", _mut_upsample_no_scale),
    ("bilinear", _mut_bilinear_swap),
    ("reduce", _mut_reduce_no_clamp),
    ("normalize", _mut_normalize_one_pass_wrong),
]


@pytest.mark.parametrize("name,mut", MUTATIONS, ids=[m[1].__name__ for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, mut):
    monkeypatch.setattr(O, name, mut)
    assert _caught(), f"mutation {mut.__name__} of {name} was not caught by any pin"
