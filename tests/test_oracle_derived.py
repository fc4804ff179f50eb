"""Pins of the oracle's live derived quantities (CPU only): vorticity against
numpy.gradient and closed-form fields, the recirculation area against a
scalar loop, probes against exact bilinear cases."""
import numpy as np
import pytest
import torch

import oracle

RNG = np.random.default_rng(77)


@pytest.mark.parametrize("shape", [(2, 2), (3, 7), (16, 5), (33, 40)])
def test_derivatives_match_numpy_gradient(shape):
    f = RNG.normal(size=shape)
    gi = np.gradient(f, axis=1, edge_order=1)
    gj = np.gradient(f, axis=0, edge_order=1)
    assert np.allclose(oracle.ddi(f).numpy(), gi, rtol=0, atol=1e-14)
    assert np.allclose(oracle.ddj(f).numpy(), gj, rtol=0, atol=1e-14)


def test_derivative_of_a_single_pixel_dimension_is_zero():
    f = RNG.normal(size=(1, 9))
    assert torch.all(oracle.ddj(f) == 0)
    assert torch.all(oracle.ddi(f.T) == 0)
    assert np.allclose(oracle.ddi(f).numpy(), np.gradient(f, axis=1, edge_order=1), atol=1e-14)


@pytest.mark.parametrize("dx,dz,dt", [(1.0, 1.0, 1.0), (0.5, 2.0, 0.01), (3.0, 0.25, 4.0)])
def test_solid_body_rotation_has_twice_the_angular_velocity(dx, dz, dt):
    # physical field U = -Om Z, V = Om X (X = i dx, Z = j dz): vorticity 2 Om everywhere
    om = 0.37
    h, w = 11, 14
    j, i = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    u = -om * (j * dz) * dt / dx
    v = om * (i * dx) * dt / dz
    got = oracle.vorticity(u, v, dx, dz, dt)
    assert torch.max(torch.abs(got - 2 * om)).item() < 1e-12


def test_pure_strain_is_irrotational_and_shear_is_not():
    h, w = 9, 12
    j, i = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    assert torch.max(torch.abs(oracle.vorticity(0.3 * i, -0.3 * j))).item() < 1e-14
    assert torch.max(torch.abs(oracle.vorticity(0.25 * j, 0 * j) + 0.25)).item() < 1e-14


def test_vorticity_is_zero_on_masked_pixels():
    u, v = RNG.normal(size=(8, 8)), RNG.normal(size=(8, 8))
    mask = RNG.integers(0, 2, (8, 8)).astype(np.uint8)
    full = oracle.vorticity(u, v)
    got = oracle.vorticity(u, v, mask=mask)
    m = torch.as_tensor(mask != 0)
    assert torch.equal(got[m], full[m]) and torch.all(got[~m] == 0)


def test_recirculation_area_matches_a_scalar_loop():
    u = RNG.normal(size=(13, 17))
    u[3, 4] = 0.0
    u[5, 6] = -0.0
    mask = RNG.integers(0, 2, u.shape).astype(np.uint8)
    for sign in (1, -1):
        n = 0
        for y in range(u.shape[0]):
            for x in range(u.shape[1]):
                if mask[y, x] and sign * u[y, x] < 0:
                    n += 1
        area, cnt = oracle.recirculation_area(u, 0.5, 0.25, mask=mask, sign=sign)
        assert cnt == n and area == n * 0.5 * 0.25
    # every unmasked pixel is negative, positive or zero
    a, _ = oracle.recirculation_area(u, sign=1)
    b, _ = oracle.recirculation_area(u, sign=-1)
    assert a + b + int(np.sum(u == 0)) == u.size


def test_probes_exact_at_pixels_and_on_affine_fields():
    h, w = 10, 12
    j, i = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    u = 0.3 * i - 0.2 * j + 1.0
    v = -0.1 * i + 0.4 * j
    pts = np.array([[0, 0], [3, 4], [11, 9], [2.25, 7.5], [10.75, 0.5], [-3, 2], [20, 30]], dtype=float)
    got = oracle.probes(u, v, pts, dx=2.0, dz=0.5, dt=0.1).numpy()
    xc = np.clip(pts[:, 0], 0, w - 1)
    yc = np.clip(pts[:, 1], 0, h - 1)
    assert np.allclose(got[:, 0], (0.3 * xc - 0.2 * yc + 1.0) * 2.0 / 0.1, atol=1e-12)
    assert np.allclose(got[:, 1], (-0.1 * xc + 0.4 * yc) * 0.5 / 0.1, atol=1e-12)


# ---------------------------------------------------------------- planted mistakes

from oracle import ofv_derived as D  # noqa: E402


def _checks():
    """Fast versions of the pins above; True when all pass."""
    ok = True
    f = np.random.default_rng(5).normal(size=(6, 7))
    ok &= np.allclose(D.ddi(f).numpy(), np.gradient(f, axis=1, edge_order=1), atol=1e-14)
    ok &= np.allclose(D.ddj(f).numpy(), np.gradient(f, axis=0, edge_order=1), atol=1e-14)
    j, i = np.meshgrid(np.arange(7.0), np.arange(9.0), indexing="ij")
    ok &= torch.max(torch.abs(D.vorticity(-0.5 * j * 2.0 / 0.5, 0.5 * i * 0.5 / 2.0, 0.5, 2.0) - 1.0)).item() < 1e-12
    u = np.array([[-1.0, 0.0, 2.0], [-0.0, -3.0, 1.0]])
    ok &= D.recirculation_area(u)[1] == 2 and D.recirculation_area(u, sign=-1)[1] == 2
    ok &= np.allclose(D.probes(i, j, [[2.5, 1.25]]).numpy(), [[2.5, 1.25]], atol=1e-12)
    return bool(ok)


def test_unmutated_derived_oracle_passes():
    assert _checks()


def _mut_forward_difference(f):
    f = D._t(f)
    d = torch.zeros_like(f)
    if f.shape[1] >= 2:
        d[:, :-1] = f[:, 1:] - f[:, :-1]
        d[:, -1] = f[:, -1] - f[:, -2]
    return d


def _mut_vorticity_sign(u, v, dx=1.0, dz=1.0, dt=1.0, mask=None):
    u, v = D._t(u), D._t(v)
    return (dz / dx) / dt * D.ddi(v) + (dx / dz) / dt * D.ddj(u)


def _mut_vorticity_swapped_ratio(u, v, dx=1.0, dz=1.0, dt=1.0, mask=None):
    u, v = D._t(u), D._t(v)
    return (dx / dz) / dt * D.ddi(v) - (dz / dx) / dt * D.ddj(u)


def _mut_area_non_strict(u, dx=1.0, dz=1.0, mask=None, sign=1):
    n = int(((sign * D._t(u)) <= 0).sum().item())
    return n * dx * dz, n


def _mut_probe_unscaled(u, v, xy, dx=1.0, dz=1.0, dt=1.0):
    p = D._t(xy).reshape(-1, 2)
    return torch.stack([D.bilinear(D._t(u), p[:, 1], p[:, 0]), D.bilinear(D._t(v), p[:, 1], p[:, 0])], dim=1)


@pytest.mark.parametrize("name,mut", [("ddi", _mut_forward_difference), ("vorticity", _mut_vorticity_sign),
                                      ("vorticity", _mut_vorticity_swapped_ratio),
                                      ("recirculation_area", _mut_area_non_strict),
                                      ("probes", _mut_probe_unscaled)],
                         ids=["forward_difference", "vorticity_sign", "swapped_ratio", "area_non_strict",
                              "probe_xy_swapped"])
def test_planted_mistake_in_derived_oracle_is_caught(monkeypatch, name, mut):
    monkeypatch.setattr(D, name, mut)
    assert not _checks(), f"mutation {mut.__name__} of {name} was not caught"
