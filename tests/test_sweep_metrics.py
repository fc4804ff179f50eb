"""Pins of the accuracy metrics of the parameter sweep (CPU): the unfolding
grid, and Psi of Eq. (psi_metric) on fields whose answer is known in closed
form."""
import math

import numpy as np
import torch

import synth
from synth import metrics as M


def test_unfolding_grid_covers_half_a_turn_with_one_pixel_arcs():
    for r in (12.0, 50.0, 300.0):
        x, y, s = M.unfolding_grid(100.0, 80.0, r)
        n_theta, n_r = x.shape
        assert n_r == 2 * int(r) + 1 and s[0, 0] == -int(r) and s[0, -1] == int(r)
        dth = math.pi / n_theta
        assert r * dth <= 1.0 and r * math.pi / (n_theta - 1) > 1.0
        assert np.allclose(np.hypot(x - 100.0, y - 80.0), np.abs(s))


def test_psi_of_a_zero_field_is_the_mean_theoretical_magnitude():
    v = synth.Rankine(60.0, 64.0, 12.0, 8.0)
    flows = torch.zeros((1, 2, 128, 128), dtype=torch.float64)
    r_max = 24.0
    s = np.arange(-24, 25, dtype=np.float64)
    expect = float(np.mean(v.magnitude_profile(np.abs(s))))
    assert abs(M.psi(flows, v, r_max).item() - expect) < 1e-12


def test_psi_of_a_uniform_field_above_the_profile():
    v = synth.Rankine(60.0, 64.0, 12.0, 8.0)
    c = 10.0                                   # above every theoretical magnitude (max 2 r sin(D / 2R) < 8)
    flows = torch.zeros((2, 2, 128, 128), dtype=torch.float64)
    flows[0, 0] = c
    flows[1, 0] = c * 0.6
    flows[1, 1] = -c * 0.8
    s = np.arange(-24, 25, dtype=np.float64)
    expect = c - float(np.mean(v.magnitude_profile(np.abs(s))))
    got = M.psi(flows, v, 24.0)
    assert torch.max(torch.abs(got - expect)).item() < 1e-12


def test_bilinear_sampling_is_exact_on_linear_magnitudes():
    h, w = 40, 50
    yy, xx = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    plane = torch.as_tensor(1.0 + 0.25 * xx + 0.5 * yy)[None]
    x = torch.as_tensor([[3.25, 10.5], [48.0, 0.0]], dtype=torch.float64)
    y = torch.as_tensor([[7.75, 0.5], [38.5, 39.0]], dtype=torch.float64)
    got = M._bilinear_many(plane, x, y)[0]
    assert torch.max(torch.abs(got - (1.0 + 0.25 * x + 0.5 * y))).item() < 1e-12


def test_mean_endpoint_error_excludes_the_border():
    gt = torch.zeros((2, 10, 10), dtype=torch.float64)
    f = torch.zeros((1, 2, 10, 10), dtype=torch.float64)
    f[0, 0, 0, :] = 100.0                     # only in the border band
    f[0, 1, 2:8, 2:8] = 3.0
    f[0, 0, 2:8, 2:8] = 4.0
    assert M.mean_endpoint_error(f, gt, 2).item() == 5.0


def test_paper_best_settings_fixture_shows_kr_falling_with_d_over_r():
    """The transcribed table: window radius falls as the displacement gradient D/R grows."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
    rows = np.array(d["rankine_best_settings"]["rows"], dtype=float)
    assert rows.shape == (24, 7)
    dr = rows[:, 1] / rows[:, 0]
    kr = rows[:, 3]
    rank = lambda a: np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(float)
    rho = np.corrcoef(rank(dr), rank(kr))[0, 1]
    assert rho < -0.6
