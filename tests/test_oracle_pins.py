"""Pins of the FP64 oracle against things other than itself (CPU only).

Each stage is checked against brute-force scalar loops, closed forms,
invariants that the mathematics fixes, or a textbook routine, and the
whole pipeline against the paper's printed accuracy figures.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import bruteforce as bf

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
RNG = np.random.default_rng(1234)


def T(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------- normalisation

@pytest.mark.parametrize("nr", [1, 2])
def test_normalize_matches_bruteforce(nr):
    img = RNG.uniform(0, 1, (9, 7))
    got = oracle.normalize(T(img), nr, 1e-4).numpy()
    ref = bf.bf_normalize(img, nr, 1e-4)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_normalize_constant_is_zero():
    # dyadic constant: the window means are exact, so N is exactly 0
    img = torch.full((11, 13), 0.375, dtype=torch.float64)
    assert torch.count_nonzero(oracle.normalize(img, 2, 1e-4)) == 0
    # any constant: zero up to the rounding of the mean
    img = torch.full((11, 13), 0.37, dtype=torch.float64)
    assert torch.max(oracle.normalize(img, 2, 1e-4).abs()) < 1e-12


def test_normalize_samuelson_bound():
    # |z| <= sqrt(n - 1) for a z-score within an n-sample window
    img = T(RNG.uniform(0, 1, (12, 10)))
    nr = 2
    n = oracle.window_sum(torch.ones_like(img), nr)
    z = oracle.normalize(img, nr, 0.0)
    assert torch.all(z.abs() <= torch.sqrt(n - 1) + 1e-12)


def test_normalize_affine_identity():
    # N(a I + b; eps a^2) == N(I; eps)
    img = T(RNG.uniform(0, 1, (10, 10)))
    a, b, eps = 3.5, -0.25, 1e-4
    lhs = oracle.normalize(a * img + b, 1, eps * a * a)
    rhs = oracle.normalize(img, 1, eps)
    assert torch.max((lhs - rhs).abs()) < 1e-12


def test_intensity_scaling():
    f = np.array([[0, 4095], [2048, 1]], dtype=np.uint16)
    i = oracle.intensity(f, 12).numpy()
    assert i[0, 0] == 0.0 and i[0, 1] == 1.0 and abs(i[1, 0] - 2048 / 4095) < 1e-16


# ---------------------------------------------------------------- pyramid

@pytest.mark.parametrize("shape", [(9, 7), (8, 8), (5, 12), (1, 6)])
def test_reduce_matches_bruteforce(shape):
    p = RNG.normal(size=shape)
    assert np.max(np.abs(oracle.reduce(T(p)).numpy() - bf.bf_reduce(p))) < 1e-12


def test_reduce_preserves_constants_exactly():
    p = torch.full((17, 9), -1.75, dtype=torch.float64)
    r = oracle.reduce(p)
    assert r.shape == (9, 5) and torch.all(r == -1.75)


def test_reduce_maps_ramps_to_ramps_at_2x():
    h, w = 20, 24
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    p = 0.3 * xx - 0.7 * yy + 2.0
    r = oracle.reduce(T(p)).numpy()
    ys, xs = np.mgrid[0:r.shape[0], 0:r.shape[1]].astype(np.float64)
    expect = 0.3 * 2 * xs - 0.7 * 2 * ys + 2.0
    assert np.max(np.abs(r[1:-1, 1:-1] - expect[1:-1, 1:-1])) < 1e-12


# ---------------------------------------------------------------- bilinear / gradient / window

def test_bilinear_exact_at_integers_and_affine_inside():
    p = RNG.normal(size=(6, 8))
    yy, xx = np.mgrid[0:6, 0:8].astype(np.float64)
    assert torch.equal(oracle.bilinear(T(p), T(xx), T(yy)), T(p))
    a = 0.5 * xx + 1.25 * yy - 3.0
    xs = RNG.uniform(0, 7, 50)
    ys = RNG.uniform(0, 5, 50)
    got = oracle.bilinear(T(a), T(xs), T(ys)).numpy()
    assert np.max(np.abs(got - (0.5 * xs + 1.25 * ys - 3.0))) < 1e-12


def test_bilinear_clamps_and_is_continuous():
    p = RNG.normal(size=(5, 5))
    pt = T(p)
    # clamping: outside samples equal the border value
    assert oracle.bilinear(pt, T([-3.0]), T([2.0])).item() == p[2, 0]
    assert oracle.bilinear(pt, T([2.0]), T([9.0])).item() == p[4, 2]
    # continuity across an integer crossing
    e = 1e-9
    left = oracle.bilinear(pt, T([2.0 - e]), T([1.3])).item()
    right = oracle.bilinear(pt, T([2.0 + e]), T([1.3])).item()
    assert abs(left - right) < 1e-7
    assert abs(left - bf.bf_bilinear(p, 2.0 - e, 1.3)) < 1e-12


def test_central_gradient_exact_for_quadratics():
    h, w = 9, 11
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    s = 0.2 * xx * xx - 0.1 * xx * yy + 0.3 * yy * yy + 0.5 * xx - 0.7 * yy
    gx, gy = oracle.central_gradient(T(s))
    ex = 0.4 * xx - 0.1 * yy + 0.5
    ey = -0.1 * xx + 0.6 * yy - 0.7
    assert np.max(np.abs(gx.numpy()[:, 1:-1] - ex[:, 1:-1])) < 1e-12
    assert np.max(np.abs(gy.numpy()[1:-1, :] - ey[1:-1, :])) < 1e-12
    # clamped border: one-sided difference halved
    assert abs(gx[0, 0].item() - 0.5 * (s[0, 1] - s[0, 0])) < 1e-15


@pytest.mark.parametrize("r", [1, 3])
def test_window_sum_bruteforce_and_counts(r):
    x = RNG.normal(size=(7, 9))
    got = oracle.window_sum(T(x), r).numpy()
    h, w = x.shape
    for y in range(h):
        for xx in range(w):
            ref = x[max(0, y - r):y + r + 1, max(0, xx - r):xx + r + 1].sum()
            assert abs(got[y, xx] - ref) < 1e-12
    cnt = oracle.window_sum(torch.ones(7, 9, dtype=torch.float64), r).numpy()
    assert cnt[3, 4] == min(2 * r + 1, 7) * min(2 * r + 1, 9)
    assert cnt[0, 0] == (r + 1) * (r + 1)


def test_window_sum_self_adjoint():
    a = T(RNG.normal(size=(8, 10)))
    b = T(RNG.normal(size=(8, 10)))
    lhs = torch.sum(oracle.window_sum(a, 2) * b)
    rhs = torch.sum(a * oracle.window_sum(b, 2))
    assert abs((lhs - rhs).item()) < 1e-11


# ---------------------------------------------------------------- one GN step

def _tiny_levels(h=8, w=8, seed=0):
    rng = np.random.default_rng(seed)
    p0 = rng.normal(size=(h, w))
    p1 = rng.normal(size=(h, w))
    u = rng.uniform(-1.5, 1.5, (h, w))
    v = rng.uniform(-1.5, 1.5, (h, w))
    return p0, p1, u, v


@pytest.mark.parametrize("kr", [1, 2])
def test_gn_iteration_matches_per_window_solve(kr):
    p0, p1, u, v = _tiny_levels()
    un, vn = oracle.gn_iteration(T(p0), T(p1), T(u), T(v), kr, 1e-3, 1e-9)
    ru, rv = bf.bf_gn_iteration(p0, p1, u, v, kr, 1e-3, 1e-9)
    assert np.max(np.abs(un.numpy() - ru)) < 1e-10
    assert np.max(np.abs(vn.numpy() - rv)) < 1e-10


def test_gn_solve_equals_damped_lstsq():
    # Cramer's rule == numpy lstsq on [G; sqrt(lam) I] V = [b; sqrt(lam) V(m)]
    p0, p1, u, v = _tiny_levels(seed=3)
    kr, rr, ra = 1, 1e-2, 1e-6
    terms = []
    un, vn = oracle.gn_iteration(T(p0), T(p1), T(u), T(v), kr, rr, ra, terms=terms)
    gx, gy, b = terms[0].gx.numpy(), terms[0].gy.numpy(), terms[0].b.numpy()
    h, w = p0.shape
    for (y, x) in [(0, 0), (3, 4), (7, 7), (5, 1)]:
        ys = slice(max(0, y - kr), y + kr + 1)
        xs = slice(max(0, x - kr), x + kr + 1)
        a = np.stack([gx[ys, xs].ravel(), gy[ys, xs].ravel()], 1)
        lam = rr * np.sum(a * a) + ra
        A = np.vstack([a, math.sqrt(lam) * np.eye(2)])
        rhs = np.concatenate([b[ys, xs].ravel(), math.sqrt(lam) * np.array([u[y, x], v[y, x]])])
        sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
        assert abs(sol[0] - un[y, x].item()) < 1e-10 and abs(sol[1] - vn[y, x].item()) < 1e-10


def test_textbook_symmetric_lk_without_damping():
    # reg = 0, V = 0: one step solves (sum G G^T) V = -sum G T
    p0, p1, _, _ = _tiny_levels(seed=5)
    z = torch.zeros(8, 8, dtype=torch.float64)
    terms = []
    un, vn = oracle.gn_iteration(T(p0), T(p1), z, z, 2, 0.0, 0.0, terms=terms)
    s = 0.5 * (p0 + p1)
    t = p1 - p0
    gx = np.zeros_like(s)
    gy = np.zeros_like(s)
    gx[:, 1:-1] = 0.5 * (s[:, 2:] - s[:, :-2])
    gx[:, 0] = 0.5 * (s[:, 1] - s[:, 0])
    gx[:, -1] = 0.5 * (s[:, -1] - s[:, -2])
    gy[1:-1] = 0.5 * (s[2:] - s[:-2])
    gy[0] = 0.5 * (s[1] - s[0])
    gy[-1] = 0.5 * (s[-1] - s[-2])
    y, x = 4, 4
    sl = (slice(2, 7), slice(2, 7))
    A = np.array([[np.sum(gx[sl] ** 2), np.sum(gx[sl] * gy[sl])],
                  [np.sum(gx[sl] * gy[sl]), np.sum(gy[sl] ** 2)]])
    c = -np.array([np.sum(gx[sl] * t[sl]), np.sum(gy[sl] * t[sl])])
    sol = np.linalg.solve(A, c)
    assert abs(sol[0] - un[y, x].item()) < 1e-10 and abs(sol[1] - vn[y, x].item()) < 1e-10


# ---------------------------------------------------------------- whole pipeline, brute force

@pytest.mark.parametrize("levels,kr,it", [(1, 1, 1), (1, 2, 3), (2, 1, 3), (2, 2, 1)])
def test_pipeline_matches_bruteforce_8x8(levels, kr, it):
    rng = np.random.default_rng(100 + 10 * levels + kr + it)
    i0 = rng.uniform(0, 1, (8, 8))
    i1 = rng.uniform(0, 1, (8, 8))
    v0 = rng.uniform(-1, 1, (2, 8, 8))
    prm = {"num_levels": levels, "kernel_radius": kr, "iterations": it, "norm_radius": 1,
           "norm_eps": 1e-4, "reg_rel": 1e-3, "reg_abs": 1e-9}
    got = oracle.compute_flow(i0, i1, prm, bit_depth0=0,
                              flow_init=v0).numpy()
    ref = bf.bf_compute_flow(i0, i1, levels, kr, it, 1, 1e-4, 1e-3, 1e-9, flow_init=v0)
    assert np.max(np.abs(got - ref)) < 1e-10


def test_pipeline_matches_bruteforce_odd_sizes_integer_frames():
    rng = np.random.default_rng(7)
    f0 = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    f1 = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    prm = {"num_levels": 2, "kernel_radius": 2, "iterations": 2, "norm_radius": 2}
    got = oracle.compute_flow(f0, f1, prm, bit_depth0=8).numpy()
    ref = bf.bf_compute_flow(f0 / 255.0, f1 / 255.0, 2, 2, 2, 2, 1e-4, 1e-3, 1e-9)
    assert np.max(np.abs(got - ref)) < 1e-10


# ---------------------------------------------------------------- invariants

PRM_SMALL = {"num_levels": 2, "kernel_radius": 3, "iterations": 2, "norm_radius": 1}


def _pair64(seed=11, n=48):
    pair = synth.make_pair(n, n, synth.Translation(0.8, -0.4), fwhm=2.5, ppp=0.1, seed=seed,
                           bit_depth=8, noise=2.0)
    return pair.frame0, pair.frame1


def test_identical_frames_give_exactly_zero_flow():
    f0, _ = _pair64()
    out = oracle.compute_flow(f0, f0, PRM_SMALL, bit_depth0=8)
    assert torch.count_nonzero(out) == 0


def test_frame_swap_antisymmetry_exact():
    f0, f1 = _pair64()
    a = oracle.compute_flow(f0, f1, PRM_SMALL, bit_depth0=8)
    b = oracle.compute_flow(f1, f0, PRM_SMALL, bit_depth0=8)
    assert torch.equal(a, -b)


def test_transpose_equivariance():
    f0, f1 = _pair64(n=40)
    a = oracle.compute_flow(f0, f1, PRM_SMALL, bit_depth0=8)
    b = oracle.compute_flow(np.ascontiguousarray(f0.T), np.ascontiguousarray(f1.T), PRM_SMALL,
                            bit_depth0=8)
    assert torch.max((a[0] - b[1].T).abs()) < 1e-11
    assert torch.max((a[1] - b[0].T).abs()) < 1e-11


def _shifted_pair(tx, ty, n=64, margin=8, seed=21):
    tex = synth.make_texture(n, n, fwhm=2.5, ppp=0.1, seed=seed, margin=margin)
    f0 = tex[margin:margin + n, margin:margin + n]
    f1 = tex[margin - ty:margin - ty + n, margin - tx:margin - tx + n]   # f1(x) = f0(x - t)
    return f0, f1


def test_integer_translation_is_an_exact_fixed_point():
    tx, ty = 2, -1
    f0, f1 = _shifted_pair(tx, ty)
    n = f0.shape[0]
    init = np.stack([np.full((n, n), float(tx)), np.full((n, n), float(ty))])
    prm = {"num_levels": 1, "kernel_radius": 3, "iterations": 1, "norm_radius": 0}
    out = oracle.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init).numpy()
    b = 3 + 2 + 2
    assert np.max(np.abs(out[0, b:-b, b:-b] - tx)) < 1e-12
    assert np.max(np.abs(out[1, b:-b, b:-b] - ty)) < 1e-12


def test_integer_translation_recovered_from_zero():
    # t is an exact fixed point; the Jacobi Gauss-Newton sweep converges to it
    # geometrically in IT (the interior mean error at least halves per
    # doubling of IT) and reaches 1e-3 px on average by IT = 16
    tx, ty = 2, -1
    f0, f1 = _shifted_pair(tx, ty)
    b = 12
    means = []
    for it in (4, 8, 16):
        prm = {"num_levels": 2, "kernel_radius": 3, "iterations": it, "norm_radius": 1}
        out = oracle.compute_flow(f0, f1, prm, bit_depth0=0).numpy()
        means.append(np.hypot(out[0] - tx, out[1] - ty)[b:-b, b:-b].mean())
    assert means[1] < 0.5 * means[0] and means[2] < 0.5 * means[1]
    assert means[2] < 1e-3


@pytest.mark.parametrize("t", [(0.35, -0.2), (1.6, 0.7)])
@pytest.mark.parametrize("nr", [0, 1])
def test_subpixel_translation_accuracy(t, nr):
    pair = synth.make_pair(96, 96, synth.Translation(*t), fwhm=2.5, ppp=0.1, seed=31, bit_depth=0)
    prm = {"num_levels": 2, "kernel_radius": 4, "iterations": 4, "norm_radius": nr}
    out = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=0)
    err = oracle.endpoint_error(out, pair.gt).numpy()[16:-16, 16:-16]
    # without normalisation only the bilinear interpolation bias remains: at
    # least as good as the paper's best Rankine <Err> (0.048 px); the 3x3
    # z-score is not shift-equivariant at sub-pixel offsets, so with NR = 1
    # the gate is the top of the paper's Rankine range
    bound = 0.05 if nr == 0 else GOLDEN["rankine_mean_err_px"]["max"]
    assert err.mean() <= bound
    assert err.max() < 0.5


def test_pyramid_capacity_rule():
    # PSL 0 handles ~1 px, PSL 1 up to ~4 px (section 'Post-processing (offline) performances')
    cap = GOLDEN["psl_capacity_px"]
    d = 3.5
    assert float(cap["1"]) >= d > float(cap["0"])
    pair = synth.make_pair(128, 128, synth.Translation(d, 0.0), fwhm=2.5, ppp=0.1, seed=41, bit_depth=0)
    b = 24
    errs = {}
    for levels in (1, 2):
        prm = {"num_levels": levels, "kernel_radius": 4, "iterations": 4, "norm_radius": 1}
        out = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=0)
        errs[levels] = oracle.endpoint_error(out, pair.gt).numpy()[b:-b, b:-b].mean()
    assert errs[2] < 0.1 < 0.5 < errs[1]


# ---------------------------------------------------------------- closed-form Rankine (workload rankine_256)

def test_rankine_accuracy_within_paper_range():
    pair, prm = synth.config_rankine_256()
    out = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=8)
    err = oracle.endpoint_error(out, pair.gt).numpy()
    b = prm["kernel_radius"] * 2 ** (prm["num_levels"] - 1)
    inner = err[b:-b, b:-b]
    assert inner.mean() <= GOLDEN["rankine_mean_err_px"]["max"]
    # D/R = 3/32 is far below the ~0.7 limit: every vector is sub-pixel
    assert 3.0 / 32.0 < GOLDEN["subpixel_limit_D_over_R"]["value"]
    assert inner.max() < 1.0
    # theta-averaged radial profile: peak within 5 % of the theoretical
    # profile sampled the same way (section 'Rankine vortex - Resolution of
    # small scales': maxima slightly underestimated, within 5 %)
    h, w = err.shape
    c = (h - 1) / 2.0
    yy, xx = np.mgrid[0:h, 0:w]
    r = np.hypot(xx - c, yy - c)
    mag = np.hypot(out[0].numpy(), out[1].numpy())
    mag_th = np.hypot(pair.gt[0], pair.gt[1])
    bins = np.arange(0, 100, 1.0)
    idx = np.digitize(r, bins)
    prof = np.array([mag[idx == i].mean() for i in range(1, len(bins))])
    prof_th = np.array([mag_th[idx == i].mean() for i in range(1, len(bins))])
    assert abs(prof.max() - prof_th.max()) / prof_th.max() < 0.05
    assert abs(int(np.argmax(prof)) - int(np.argmax(prof_th))) <= 1


def test_endpoint_error_definition():
    f = np.zeros((2, 2, 2))
    g = np.zeros((2, 2, 2))
    g[0, 0, 0], g[1, 0, 0] = 3.0, 4.0
    e = oracle.endpoint_error(f, g).numpy()
    assert e[0, 0] == 5.0 and e[1, 1] == 0.0


# ---------------------------------------------------------------- storage rounding (precision floor, not the method)

@pytest.mark.parametrize("kind,ulp", [("f16", 2.0 ** -10), ("bf16", 2.0 ** -7)])
def test_round_plane_is_round_to_nearest_even(kind, ulp):
    # values around 1 where the ulp is known: halfway cases go to the even neighbour
    x = T([1.0, 1.0 + ulp / 2, 1.0 + 1.5 * ulp, 1.0 + 0.75 * ulp, -(1.0 + ulp / 2), 1.0 + 0.25 * ulp])
    want = [1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -1.0, 1.0]
    assert oracle.ofv_oracle.round_plane(x, kind).tolist() == want
    assert oracle.ofv_oracle.round_plane(x, None) is x


def test_plane_rounding_applies_to_every_level():
    pair, prm = synth.config_rankine_256()
    tr = oracle.Trace()
    oracle.compute_flow(pair.frame0, pair.frame1, dict(prm, iterations=1), bit_depth0=8, trace=tr, plane_round="f16")
    for lev, p in enumerate(tr.levels0):
        assert torch.equal(p.half().double(), p), lev          # representable in binary16
        if lev:                                                # REDUCE read the rounded finer level
            assert torch.equal(oracle.reduce(tr.levels0[lev - 1]).half().double(), p), lev


def test_float32_planes_stay_within_fp32_tolerance():
    # storing the planes in binary32 moves the result by far less than the
    # 1e-3 px that the float32 implementation is held to
    pair, prm = synth.config_rankine_256()
    ref = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=8)
    got = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=8, plane_round="f32")
    assert 0 < torch.max(torch.abs(got - ref)).item() < 1e-4


# ---------------------------------------------------------------- forward-additive estimator (R24)

@pytest.mark.parametrize("levels,kr,it", [(1, 1, 1), (1, 2, 3), (2, 1, 3), (2, 2, 2)])
def test_forward_additive_matches_bruteforce_8x8(levels, kr, it):
    rng = np.random.default_rng(300 + 10 * levels + kr + it)
    i0 = rng.uniform(0, 1, (8, 8))
    i1 = rng.uniform(0, 1, (8, 8))
    v0 = rng.uniform(-1, 1, (2, 8, 8))
    prm = {"num_levels": levels, "kernel_radius": kr, "iterations": it, "norm_radius": 1,
           "estimator": "forward_additive"}
    got = oracle.compute_flow(i0, i1, prm, bit_depth0=0, flow_init=v0).numpy()
    ref = bf.bf_compute_flow(i0, i1, levels, kr, it, 1, 1e-4, 1e-3, 1e-9, flow_init=v0, forward_additive=True)
    assert np.max(np.abs(got - ref)) < 1e-10
    sym = oracle.compute_flow(i0, i1, dict(prm, estimator="symmetric"), bit_depth0=0, flow_init=v0).numpy()
    assert np.max(np.abs(got - sym)) > 1e-3      # a different estimator


def _check_fa_fixed_point():
    tx, ty = 2, -1
    f0, f1 = _shifted_pair(tx, ty)
    n = f0.shape[0]
    init = np.stack([np.full((n, n), float(tx)), np.full((n, n), float(ty))])
    prm = {"num_levels": 1, "kernel_radius": 3, "iterations": 1, "norm_radius": 0, "estimator": "forward_additive"}
    out = oracle.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init).numpy()
    b = 3 + 2 + 2
    return max(np.max(np.abs(out[0, b:-b, b:-b] - tx)), np.max(np.abs(out[1, b:-b, b:-b] - ty)))


def test_forward_additive_integer_translation_is_an_exact_fixed_point():
    # f1(k + t) = f0(k): the full-step warp of the second frame matches the first exactly
    assert _check_fa_fixed_point() < 1e-12


def test_textbook_forward_additive_lk_without_damping():
    # reg = 0, V = 0: one step solves (sum G G^T) V = -sum G (I1 - I0), G the gradient of I1
    p0, p1, _, _ = _tiny_levels(seed=6)
    z = torch.zeros(8, 8, dtype=torch.float64)
    un, vn = oracle.gn_iteration(T(p0), T(p1), z, z, 2, 0.0, 0.0, estimator="forward_additive")
    gy, gx = np.gradient(p1, edge_order=1)
    gx[:, 0] *= 0.5
    gx[:, -1] *= 0.5
    gy[0] *= 0.5
    gy[-1] *= 0.5     # central differences with clamped indices halve the one-sided edge steps
    t = p1 - p0
    y, x = 4, 4
    sl = (slice(2, 7), slice(2, 7))
    A = np.array([[np.sum(gx[sl] ** 2), np.sum(gx[sl] * gy[sl])],
                  [np.sum(gx[sl] * gy[sl]), np.sum(gy[sl] ** 2)]])
    c = -np.array([np.sum(gx[sl] * t[sl]), np.sum(gy[sl] * t[sl])])
    sol = np.linalg.solve(A, c)
    assert abs(sol[0] - un[y, x].item()) < 1e-10 and abs(sol[1] - vn[y, x].item()) < 1e-10


def test_planted_half_step_in_forward_additive_is_caught(monkeypatch):
    from oracle import ofv_oracle as O

    def mut(p0, p1, u, v):
        h, w = p0.shape
        yy, xx = torch.meshgrid(torch.arange(h, dtype=O.DT), torch.arange(w, dtype=O.DT), indexing="ij")
        w1 = O.bilinear(p1, xx + 0.5 * u, yy + 0.5 * v)
        return w1, w1 - p0
    monkeypatch.setattr(O, "warp_terms_forward", mut)
    assert _check_fa_fixed_point() > 1e-3


# ---------------------------------------------------------------- increment-form update (R25)

@pytest.mark.parametrize("estimator", ["symmetric", "forward_additive"])
@pytest.mark.parametrize("levels,kr,it", [(1, 1, 1), (1, 2, 3), (2, 1, 3), (2, 2, 2)])
def test_increment_update_matches_bruteforce_8x8(estimator, levels, kr, it):
    """The oracle's increment update against the brute force, which stacks one row per
    window pixel in the unknown step and its damping rows and hands them to numpy."""
    rng = np.random.default_rng(400 + 10 * levels + kr + it)
    i0 = rng.uniform(0, 1, (8, 8))
    i1 = rng.uniform(0, 1, (8, 8))
    v0 = rng.uniform(-1, 1, (2, 8, 8))
    prm = {"num_levels": levels, "kernel_radius": kr, "iterations": it, "norm_radius": 1,
           "estimator": estimator, "update": "increment"}
    got = oracle.compute_flow(i0, i1, prm, bit_depth0=0, flow_init=v0).numpy()
    ref = bf.bf_compute_flow(i0, i1, levels, kr, it, 1, 1e-4, 1e-3, 1e-9, flow_init=v0,
                             forward_additive=estimator == "forward_additive", increment=True)
    # relative: on random 8x8 pairs the forward-additive increment iteration runs away (|V| ~ 10 after
    # a few steps) and amplifies the different rounding orders of the two computations; a slip in the
    # formula moves the result by O(1) (test_planted_mistakes_in_the_increment_step_are_caught)
    tol = 1e-10 if estimator == "symmetric" else 1e-8
    assert np.max(np.abs(got - ref) / (1.0 + np.abs(ref))) < tol
    cons = oracle.compute_flow(i0, i1, dict(prm, update="consistent"), bit_depth0=0, flow_init=v0).numpy()
    assert np.max(np.abs(got - cons)) > 1e-3      # a different update where the field varies


def test_increment_update_equals_consistent_where_the_field_is_uniform():
    """With V(k) = V(m) over every window the two linearisations coincide: exactly at V = 0 (both
    solve the same system), and up to rounding for a uniform non-zero field."""
    p0, p1, _, _ = _tiny_levels(seed=9)
    z = torch.zeros(8, 8, dtype=torch.float64)
    a = oracle.gn_iteration(T(p0), T(p1), z, z, 2, 1e-3, 1e-9, update="increment")
    b = oracle.gn_iteration(T(p0), T(p1), z, z, 2, 1e-3, 1e-9)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    cu = torch.full((8, 8), 0.7, dtype=torch.float64)
    cv = torch.full((8, 8), -0.4, dtype=torch.float64)
    for est in ("symmetric", "forward_additive"):
        a = oracle.gn_iteration(T(p0), T(p1), cu, cv, 2, 1e-3, 1e-9, estimator=est, update="increment")
        b = oracle.gn_iteration(T(p0), T(p1), cu, cv, 2, 1e-3, 1e-9, estimator=est)
        assert torch.max(torch.abs(a[0] - b[0])).item() < 1e-12
        assert torch.max(torch.abs(a[1] - b[1])).item() < 1e-12


def test_increment_update_integer_translation_is_an_exact_fixed_point():
    tx, ty = 2, -1
    f0, f1 = _shifted_pair(tx, ty)
    n = f0.shape[0]
    init = np.stack([np.full((n, n), float(tx)), np.full((n, n), float(ty))])
    prm = {"num_levels": 1, "kernel_radius": 3, "iterations": 1, "norm_radius": 0, "update": "increment"}
    out = oracle.compute_flow(f0, f1, prm, bit_depth0=0, flow_init=init).numpy()
    b = 3 + 2 + 2
    assert np.max(np.abs(out[:, b:-b, b:-b] - init[:, b:-b, b:-b])) < 1e-12


@pytest.mark.parametrize("mistake", ["no_anchor", "sign", "swapped"])
def test_planted_mistakes_in_the_increment_step_are_caught(monkeypatch, mistake):
    from oracle import ofv_oracle as O
    steps = {
        "no_anchor": lambda a, d, sxy, det, sxb, syb, u, v: ((d * sxb - sxy * syb) / det,
                                                             (a * syb - sxy * sxb) / det),
        "sign": lambda a, d, sxy, det, sxb, syb, u, v: (u - (d * sxb - sxy * syb) / det,
                                                        v - (a * syb - sxy * sxb) / det),
        "swapped": lambda a, d, sxy, det, sxb, syb, u, v: (u + (a * sxb - sxy * syb) / det,
                                                           v + (d * syb - sxy * sxb) / det),
    }
    monkeypatch.setattr(O, "increment_step", steps[mistake])
    rng = np.random.default_rng(411)
    i0 = rng.uniform(0, 1, (8, 8))
    i1 = rng.uniform(0, 1, (8, 8))
    v0 = rng.uniform(-1, 1, (2, 8, 8))
    prm = {"num_levels": 1, "kernel_radius": 1, "iterations": 1, "norm_radius": 1, "update": "increment"}
    got = O.compute_flow(i0, i1, prm, bit_depth0=0, flow_init=v0).numpy()
    ref = bf.bf_compute_flow(i0, i1, 1, 1, 1, 1, 1e-4, 1e-3, 1e-9, flow_init=v0, increment=True)
    assert np.max(np.abs(got - ref)) > 1e-6


def test_float32_arithmetic_option():
    """arith="f32" (a diagnostic floor, not the reference) runs every step in float32: on a
    well-conditioned input it stays within a few float32 roundings of the float64 reference, is
    not identical to it, and returns float64; every intermediate is float32."""
    pair, prm = synth.config_rankine_256()
    ref = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=8)
    tr = oracle.Trace()
    got = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=8, arith="f32", trace=tr)
    assert got.dtype == torch.float64
    assert all(p.dtype == torch.float32 for p in tr.levels0 + tr.levels1)
    assert all(u.dtype == torch.float32 for u, _ in tr.iterates.values())
    assert 0 < torch.max(torch.abs(got - ref)).item() < 1e-4
