"""Hand-written adjoint (ofv_compute_flow_backward) vs autograd of the FP64 oracle.

Both sides receive the same upstream gradient dL/dV = 2 (V_oracle - V_gt)
(loss = sum |V - V_gt|^2) and are compared by relative L2 error and cosine
similarity: the estimator has measure-zero kinks (bilinear weights), so an
element-wise bound does not apply to gradients.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ofv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_25924_amd as m
    m.load()
    return m


def _metrics(a, b):
    a = a.detach().double().cpu().reshape(-1)
    b = b.detach().double().cpu().reshape(-1)
    rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    cos = float(torch.dot(a, b) / (torch.linalg.norm(a) * torch.linalg.norm(b)))
    return rel, cos


def _oracle_grads(f0, f1, init, prm, g_up, bits, arith=None):
    """Autograd of the oracle; arith="f32" runs it in float32 arithmetic (a diagnostic floor)."""
    dt = torch.float32 if arith == "f32" else torch.float64
    x0 = torch.as_tensor(f0.astype(np.float64) / (1.0 if bits == 0 else 2 ** bits - 1)).to(dt).requires_grad_(True)
    x1 = torch.as_tensor(f1.astype(np.float64) / (1.0 if bits == 0 else 2 ** bits - 1)).to(dt).requires_grad_(True)
    xi = None if init is None else torch.as_tensor(init.astype(np.float64)).to(dt).requires_grad_(True)
    v = oracle.compute_flow(x0, x1, prm, bit_depth0=0, flow_init=xi, arith=arith)
    ins = [x0, x1] + ([xi] if xi is not None else [])
    gs = torch.autograd.grad(torch.sum(v * g_up.to(v.dtype)), ins)
    scale = 1.0 if bits == 0 else 1.0 / (2 ** bits - 1)
    gs = [g.double() for g in gs]
    return gs[0] * scale, gs[1] * scale, (gs[2] if xi is not None else None)


@pytest.mark.parametrize("store_all", [False, True])
@pytest.mark.parametrize("shape,levels,kr,it,nr,bits,with_init", [
    ((96, 80), 3, 3, 2, 1, 0, True),
    ((64, 64), 2, 4, 3, 2, 0, False),
    ((70, 90), 2, 2, 2, 1, 8, True),
    ((48, 48), 1, 3, 2, 0, 0, True),
    ((150, 200), 2, 7, 2, 1, 0, True),
    ((40, 56), 2, 2, 2, 3, 0, False),
])
def test_adjoint_matches_oracle_autograd(ofv, shape, levels, kr, it, nr, bits, with_init, store_all):
    say("adjoint", shape, levels, kr, it, nr, bits, with_init, "store-all" if store_all else "recompute")
    h, w = shape
    flow = synth.Rankine(w / 2 - 0.3, h / 2 + 0.2, 0.25 * min(h, w), 1.5)
    pair = synth.make_pair(h, w, flow, fwhm=2.5, ppp=0.1, seed=h + w + levels, bit_depth=bits,
                           noise=(2.0 / 255.0 if bits == 0 else 2.0))
    prm = {"num_levels": levels, "kernel_radius": kr, "iterations": it, "norm_radius": nr,
           "norm_eps": 1e-4, "reg_rel": 1e-3, "reg_abs": 1e-9}
    init = None
    if with_init:
        init = (pair.gt + np.random.default_rng(3).normal(0, 0.2, pair.gt.shape)).astype(np.float32)
    v_or = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=bits, flow_init=init)
    g_up = 2.0 * (v_or - torch.as_tensor(pair.gt))
    r0, r1, ri = _oracle_grads(pair.frame0, pair.frame1, init, prm, g_up, bits)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    gi_in = None if init is None else torch.from_numpy(init).cuda()
    g0, g1, gi = ofv.compute_flow_backward(f0, f1, dict(prm, store_all=store_all), g_up.float().cuda().contiguous(),
                                           flow_init=gi_in, bit_depth=bits or None)
    torch.cuda.synchronize()
    floor = None
    for idx, (name, got, ref) in enumerate((("frame0", g0, r0), ("frame1", g1, r1), ("flow_init", gi, ri))):
        if ref is None:
            assert got is None
            continue
        rel, cos = _metrics(got, ref)
        say(f"  {name}: rel-L2 {rel:.2e} cosine {cos:.7f}")
        assert cos >= 0.9999
        if rel > 1e-3:
            # Where the float64 gradient is a small difference of large terms (dL/dflow_init of
            # well-converged iterations: the output hardly depends on the input field), float32
            # arithmetic alone misses by more than 1e-3.  The gate is then the oracle's own error
            # when it runs the same steps in float32 arithmetic.
            if floor is None:
                floor = _oracle_grads(pair.frame0, pair.frame1, init, prm, g_up, bits, arith="f32")
            frel, _ = _metrics(floor[idx], ref)
            say(f"    float32-arithmetic oracle: rel-L2 {frel:.2e}")
            assert rel <= 1.5 * frel


def test_autograd_function(ofv):
    say("OFVFunction")
    pair = synth.make_pair(64, 72, synth.Translation(0.7, -0.4), fwhm=2.5, ppp=0.1, seed=5, bit_depth=0,
                           noise=2.0 / 255.0)
    prm = {"num_levels": 2, "kernel_radius": 3, "iterations": 2, "norm_radius": 1}
    f0 = torch.from_numpy(pair.frame0).cuda().requires_grad_(True)
    f1 = torch.from_numpy(pair.frame1).cuda().requires_grad_(True)
    init = torch.from_numpy(pair.gt.astype(np.float32)).cuda().requires_grad_(True)
    gt = torch.from_numpy(pair.gt.astype(np.float32)).cuda()
    v = ofv.OFVFunction.apply(f0, f1, init, prm, None)
    loss = torch.sum((v - gt) ** 2)
    loss.backward()
    g0, g1, gi = ofv.compute_flow_backward(f0.detach(), f1.detach(), prm, (2 * (v.detach() - gt)).contiguous(),
                                           flow_init=init.detach())
    torch.cuda.synchronize()
    for a, b in ((f0.grad, g0), (f1.grad, g1), (init.grad, gi)):
        rel, cos = _metrics(a, b)
        assert rel < 1e-5 and cos > 0.999999


def test_backward_argument_errors(ofv):
    say("backward errors")
    f = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    g = torch.zeros((2, 16, 16), dtype=torch.float32, device="cuda")
    h = ofv.Handle(16, 16, 1)
    prm = {"num_levels": 2, "kernel_radius": 2, "iterations": 2, "norm_radius": 1}
    from paper_2509_25924_amd import _lib
    from paper_2509_25924_amd.api import image_desc, params_struct
    from ctypes import byref, c_void_p
    lib = _lib.load()
    i0, i1, p = image_desc(f), image_desc(f), params_struct(prm)
    out = torch.empty((16, 16), dtype=torch.float32, device="cuda")
    st = lib.ofv_compute_flow_backward(h.ptr, byref(i0), byref(i1), byref(p), None, c_void_p(g.data_ptr()),
                                       c_void_p(out.data_ptr()), None, None)
    assert st == _lib.OFV_ERR_CAPACITY
    h.reserve_backward(2, 2)
    p16 = params_struct(dict(prm, storage="f16"))
    st = lib.ofv_compute_flow_backward(h.ptr, byref(i0), byref(i1), byref(p16), None, c_void_p(g.data_ptr()),
                                       c_void_p(out.data_ptr()), None, None)
    assert st == _lib.OFV_ERR_UNSUPPORTED
    st = lib.ofv_compute_flow_backward(h.ptr, byref(i0), byref(i1), byref(p), None, c_void_p(g.data_ptr()),
                                       c_void_p(g.data_ptr()), None, None)
    assert st == _lib.OFV_ERR_INVALID_ARG   # output overlaps grad_flow
    h.close()


def test_adjoint_matches_oracle_autograd_512(ofv):
    """The differentiation workload's shape: one 512 x 512 float pair (Rankine vortex, noise
    2/255), 3 levels, KR 4, IT 3, NR 1, loss sum |V - V_gt|^2, gradients for both frames and the
    initial field against autograd of the FP64 oracle."""
    say("adjoint 512x512")
    pair, prm = synth.config_adjoint_512(0)
    init = (pair.gt + np.random.default_rng(6).normal(0, 0.2, pair.gt.shape)).astype(np.float32)
    v_or = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=0, flow_init=init)
    g_up = 2.0 * (v_or - torch.as_tensor(pair.gt))
    r0, r1, ri = _oracle_grads(pair.frame0, pair.frame1, init, prm, g_up, 0)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    g0, g1, gi = ofv.compute_flow_backward(f0, f1, prm, g_up.float().cuda().contiguous(),
                                           flow_init=torch.from_numpy(init).cuda())
    torch.cuda.synchronize()
    for name, got, ref in (("frame0", g0, r0), ("frame1", g1, r1), ("flow_init", gi, ri)):
        rel, cos = _metrics(got, ref)
        say(f"  {name}: rel-L2 {rel:.2e} cosine {cos:.7f}")
        assert rel <= 1e-3 and cos >= 0.9999


def _pair_case(i, shape):
    h, w = shape
    flow = synth.Rankine(w / 2 + 0.4 * i, h / 2 - 0.3, 0.25 * min(h, w), 1.5 + 0.2 * i)
    return synth.make_pair(h, w, flow, fwhm=2.5, ppp=0.1, seed=70 + i, bit_depth=0, noise=2.0 / 255.0)


@pytest.mark.parametrize("store_all", [False, True])
def test_batched_backward_matches_single_pairs(ofv, store_all):
    """One batched call over pairs of uneven sizes (with and without an initial field, one without
    frame gradients) against the same pairs one at a time: the same kernels, so equal up to the
    order of the float atomics."""
    say("batched backward", "store-all" if store_all else "recompute")
    shapes = [(96, 80), (64, 130), (33, 47)]
    prm = {"num_levels": 3, "kernel_radius": 3, "iterations": 2, "norm_radius": 1, "store_all": store_all}
    pairs = [_pair_case(i, sh) for i, sh in enumerate(shapes)]
    f0 = [torch.from_numpy(p.frame0).cuda() for p in pairs]
    f1 = [torch.from_numpy(p.frame1).cuda() for p in pairs]
    gen = torch.Generator().manual_seed(11)
    gf = [torch.randn((2,) + sh, generator=gen).cuda() for sh in shapes]
    init = [torch.from_numpy(pairs[0].gt.astype(np.float32)).cuda(), None,
            torch.from_numpy(pairs[2].gt.astype(np.float32)).cuda()]
    hb = ofv.Handle(130, 96, 3)
    b0, b1, bi = ofv.compute_flow_backward_batch(f0, f1, prm, gf, flow_init=init, handle=hb)
    torch.cuda.synchronize()
    assert bi[1] is None and bi[0] is not None and bi[2] is not None
    for i in range(3):
        hs = ofv.Handle(shapes[i][1], shapes[i][0], 1)
        s0, s1, si = ofv.compute_flow_backward(f0[i], f1[i], prm, gf[i], flow_init=init[i], handle=hs)
        torch.cuda.synchronize()
        for name, a, b in (("frame0", b0[i], s0), ("frame1", b1[i], s1), ("flow_init", bi[i], si)):
            if b is None:
                assert a is None
                continue
            rel, cos = _metrics(a, b)
            say(f"  pair {i} {name}: rel-L2 {rel:.2e}")
            assert rel <= 1e-5 and cos >= 0.99999
        hs.close()
    # no frame gradients requested
    _, _, ni = ofv.compute_flow_backward_batch(f0, f1, prm, gf, flow_init=init, need_frames=False, handle=hb)
    torch.cuda.synchronize()
    rel, _ = _metrics(ni[0], bi[0])
    assert rel <= 1e-5
    hb.close()


def test_store_all_matches_recompute_512_batch(ofv):
    """The differentiation workload's shape, 16 x 512^2 float pairs (3 levels, KR 4, IT 3, NR 1), in
    one batched call in each mode: the two modes agree (their forwards run different kernels over
    the same arithmetic), and pair 0 matches the single-pair call."""
    say("store-all vs recompute, 16 x 512^2")
    n = 16
    cases = [synth.config_adjoint_512(i) for i in range(n)]
    prm = dict(cases[0][1])
    f0 = [torch.from_numpy(p.frame0).cuda() for p, _ in cases]
    f1 = [torch.from_numpy(p.frame1).cuda() for p, _ in cases]
    gt = [torch.from_numpy(p.gt.astype(np.float32)).cuda() for p, _ in cases]
    h = ofv.Handle(512, 512, n)
    outs = ofv.compute_flow_batch(f0, f1, prm, handle=h)
    gf = [(2 * (outs[i] - gt[i])).contiguous() for i in range(n)]
    r0, r1, _ = ofv.compute_flow_backward_batch(f0, f1, prm, gf, handle=h)
    s0, s1, _ = ofv.compute_flow_backward_batch(f0, f1, dict(prm, store_all=True), gf, handle=h)
    torch.cuda.synchronize()
    worst = 0.0
    for i in range(n):
        for a, b in ((s0[i], r0[i]), (s1[i], r1[i])):
            rel, cos = _metrics(a, b)
            worst = max(worst, rel)
            assert rel <= 1e-3 and cos >= 0.9999
    say(f"  worst rel-L2 store-all vs recompute {worst:.2e}")
    q0, q1, _ = ofv.compute_flow_backward(f0[0], f1[0], prm, gf[0], handle=h)
    torch.cuda.synchronize()
    for a, b in ((q0, r0[0]), (q1, r1[0])):
        rel, cos = _metrics(a, b)
        assert rel <= 1e-5
    h.close()


def test_saved_forward_reuse(ofv):
    """A forward that keeps its iterates returns the plain forward's field bit for bit, and a backward
    that reuses them equals a self-contained one; a forward on other inputs replaces them, after which
    the backward runs its own forward and still agrees.  Likewise in store-all mode."""
    say("saved forward")
    shapes = [(96, 80), (80, 96)]
    prm = {"num_levels": 3, "kernel_radius": 3, "iterations": 2, "norm_radius": 1}
    pairs = [_pair_case(i, sh) for i, sh in enumerate(shapes)]
    f0 = [torch.from_numpy(p.frame0).cuda() for p in pairs]
    f1 = [torch.from_numpy(p.frame1).cuda() for p in pairs]
    gen = torch.Generator().manual_seed(5)
    gf = [torch.randn((2,) + sh, generator=gen).cuda() for sh in shapes]
    h = ofv.Handle(96, 96, 2)
    plain = ofv.compute_flow_batch(f0, f1, prm, handle=h)
    ref = ofv.compute_flow_backward_batch(f0, f1, prm, gf, handle=h)
    saved = ofv.compute_flow_batch(f0, f1, dict(prm, save_iterates=True), handle=h)
    torch.cuda.synchronize()
    for a, b in zip(plain, saved):
        assert torch.equal(a, b)
    got = ofv.compute_flow_backward_batch(f0, f1, dict(prm, saved_forward=True), gf, handle=h)
    again = ofv.compute_flow_backward_batch(f0, f1, dict(prm, saved_forward=True), gf, handle=h)
    # another forward replaces the saved iterates: the backward runs its own forward
    ofv.compute_flow_batch([f1[0], f1[1]], [f0[0], f0[1]], prm, handle=h)
    rerun = ofv.compute_flow_backward_batch(f0, f1, dict(prm, saved_forward=True), gf, handle=h)
    torch.cuda.synchronize()
    for res in (got, again, rerun):
        for i in range(2):
            for a, b in ((res[0][i], ref[0][i]), (res[1][i], ref[1][i])):
                rel, cos = _metrics(a, b)
                assert rel <= 1e-5 and cos >= 0.99999
    # store-all: the recording forward is the estimator too, and its record serves the backward
    sa = dict(prm, store_all=True)
    rec = ofv.compute_flow_batch(f0, f1, dict(sa, save_iterates=True), handle=h)
    got_sa = ofv.compute_flow_backward_batch(f0, f1, dict(sa, saved_forward=True), gf, handle=h)
    torch.cuda.synchronize()
    for i in range(2):
        assert float((rec[i] - plain[i]).abs().max()) <= 1e-4
        for a, b in ((got_sa[0][i], ref[0][i]), (got_sa[1][i], ref[1][i])):
            rel, cos = _metrics(a, b)
            assert rel <= 1e-3 and cos >= 0.9999
    h.close()


def test_adjoint_against_central_differences_32(ofv):
    """The GPU adjoint against central differences of the FP64 oracle on 32 x 32 crops, per input
    (both frames and the initial field), along random directions: <dL/dx, d> from the GPU against
    (L(x + h d) - L(x - h d)) / 2h with h = 1e-5, L = sum(g . V).  (Central differences of the
    float32 forward itself cannot serve: at h = 1e-3 the float32 rounding of V and the bilinear
    floors crossed by the step leave them 3e-3 .. 0.5 off the exact derivative even for the oracle
    run in float32 arithmetic; at h = 1e-5 the FP64 oracle's own differences agree with its autograd
    to 4e-5.)"""
    say("adjoint vs central differences, 32x32")
    h, w = 32, 32
    flow = synth.Rankine(w / 2 - 0.3, h / 2 + 0.2, 8.0, 1.5)
    pair = synth.make_pair(h, w, flow, fwhm=2.5, ppp=0.1, seed=7, bit_depth=0, noise=2.0 / 255.0)
    prm = {"num_levels": 2, "kernel_radius": 3, "iterations": 2, "norm_radius": 1, "norm_eps": 1e-4,
           "reg_rel": 1e-3, "reg_abs": 1e-9}
    init = (pair.gt + np.random.default_rng(3).normal(0, 0.2, pair.gt.shape)).astype(np.float32)
    g = np.random.default_rng(4).normal(0, 1, (2, h, w))
    gpu = ofv.compute_flow_backward(torch.from_numpy(pair.frame0).cuda(), torch.from_numpy(pair.frame1).cuda(), prm,
                                    torch.from_numpy(g).float().cuda().contiguous(),
                                    flow_init=torch.from_numpy(init).cuda())
    torch.cuda.synchronize()
    gpu = [t.double().cpu().numpy() for t in gpu]
    base = [pair.frame0.astype(np.float64), pair.frame1.astype(np.float64), init.astype(np.float64)]
    gt = torch.from_numpy(g)
    rng = np.random.default_rng(5)
    step = 1e-5
    for which, name in enumerate(("frame0", "frame1", "flow_init")):
        for _ in range(4):
            d = rng.normal(0, 1, base[which].shape)

            def loss(sign):
                b = [x.copy() for x in base]
                b[which] = b[which] + sign * step * d
                v = oracle.compute_flow(torch.from_numpy(b[0]), torch.from_numpy(b[1]), prm, bit_depth0=0,
                                        flow_init=torch.from_numpy(b[2]))
                return float(torch.sum(v * gt))
            fd = (loss(1) - loss(-1)) / (2 * step)
            an = float(np.sum(gpu[which] * d))
            rel = abs(an - fd) / abs(fd)
            say(f"  {name}: directional derivative GPU {an:.6e} central differences {fd:.6e} rel {rel:.1e}")
            assert rel <= 2e-3


def test_adjoint_repeatable(ofv):
    """Two identical backward calls: equal up to the order in which the float atomics of the image
    gradients land (rel-L2 <= 1e-6), the flow-init gradient (no atomics) bit for bit."""
    say("adjoint repeatability")
    pair, prm = synth.config_adjoint_512(1, size=256)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    init = torch.from_numpy(pair.gt.astype(np.float32)).cuda()
    g = torch.randn((2, 256, 256), generator=torch.Generator().manual_seed(9)).cuda()
    h = ofv.Handle(256, 256, 1)
    a = ofv.compute_flow_backward(f0, f1, prm, g, flow_init=init, handle=h)
    b = ofv.compute_flow_backward(f0, f1, prm, g, flow_init=init, handle=h)
    torch.cuda.synchronize()
    for x, y in zip(a[:2], b[:2]):
        rel, _ = _metrics(x, y)
        say(f"  frame gradient: rel-L2 between runs {rel:.1e}")
        assert rel <= 1e-6
    assert torch.equal(a[2], b[2])
    h.close()
