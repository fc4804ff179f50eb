"""The seeded generators: densities, blob size, ground truth, device renderer."""
import math

import numpy as np
import torch

import synth
from synth.gpu_render import render_torch


def test_particle_density_and_fwhm():
    rng = np.random.default_rng(0)
    xs = np.array([20.3])
    ys = np.array([15.7])
    img = synth.render_particles(40, 40, xs, ys, np.array([1.0]), sigma=2.5 / synth.FWHM_PER_SIGMA)
    # total energy of a pixel-integrated blob = 2 pi sigma^2 / E(0)^2 ... check the profile peak and width
    row = img[16]
    assert abs(img.max() - img[16, 20]) < 1e-12
    half = row.max() / 2
    above = np.nonzero(row >= half)[0]
    assert 1 <= above.size <= 4          # FWHM of 2.5 px covers 2-3 pixels
    pair = synth.make_pair(64, 64, synth.Translation(0.5, 0.5), fwhm=2.5, ppp=0.1, seed=3, bit_depth=8)
    area = (64 + 2 * (1 + 4 * 2.5 / synth.FWHM_PER_SIGMA + 2)) ** 2
    assert abs(pair.n_particles - round(0.1 * area)) <= 2


def test_ground_truth_is_the_flow_at_pixel_centres():
    f = synth.Rankine(31.5, 31.5, 10.0, 2.0)
    pair = synth.make_pair(64, 64, f, fwhm=2.5, ppp=0.05, seed=4, bit_depth=8)
    yy, xx = np.mgrid[0:64, 0:64].astype(np.float64)
    u, v = f(xx, yy)
    assert np.allclose(pair.gt[0], u) and np.allclose(pair.gt[1], v)
    r = np.hypot(xx - 31.5, yy - 31.5)
    mag = np.hypot(u, v)
    assert abs(mag[r.round() == 10].max() - 2.0) < 0.05    # maximum displacement D at r = R


def test_turbulence_is_divergence_free_and_scaled():
    t = synth.Turbulence(seed=3, rms=2.0, dmax_cap=8.0, ref_h=128, ref_w=128)
    u, v = t.grid(128, 128)
    assert abs(math.sqrt(np.mean(u * u + v * v)) - 2.0) < 1e-9
    assert np.max(np.hypot(u, v)) <= 8.0
    # spectral divergence of a sum of modes with d = (dpsi/dy, -dpsi/dx) is zero: check by central differences
    e = 1e-4
    x, y = np.array([10.3, 50.7]), np.array([20.1, 90.2])
    du = (t(x + e, y)[0] - t(x - e, y)[0]) / (2 * e)
    dv = (t(x, y + e)[1] - t(x, y - e)[1]) / (2 * e)
    assert np.max(np.abs(du + dv)) < 1e-6


def test_device_renderer_matches_host_renderer_on_cpu():
    rng = np.random.default_rng(8)
    xs = rng.uniform(-3, 50, 200)
    ys = rng.uniform(-3, 40, 200)
    a = rng.uniform(0.5, 1, 200)
    sig = 2.2 / synth.FWHM_PER_SIGMA
    host = synth.render_particles(40, 50, xs, ys, a, sig)
    dev = render_torch(40, 50, xs, ys, a, sig, torch.device("cpu")).double().numpy()
    assert np.max(np.abs(host - dev)) < 1e-5
