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


def _oracle_grads(f0, f1, init, prm, g_up, bits):
    x0 = torch.as_tensor(f0.astype(np.float64) / (1.0 if bits == 0 else 2 ** bits - 1)).requires_grad_(True)
    x1 = torch.as_tensor(f1.astype(np.float64) / (1.0 if bits == 0 else 2 ** bits - 1)).requires_grad_(True)
    xi = None if init is None else torch.as_tensor(init.astype(np.float64)).requires_grad_(True)
    v = oracle.compute_flow(x0, x1, prm, bit_depth0=0, flow_init=xi)
    ins = [x0, x1] + ([xi] if xi is not None else [])
    gs = torch.autograd.grad(torch.sum(v * g_up), ins)
    scale = 1.0 if bits == 0 else 1.0 / (2 ** bits - 1)
    return gs[0] * scale, gs[1] * scale, (gs[2] if xi is not None else None)


@pytest.mark.parametrize("shape,levels,kr,it,nr,bits,with_init", [
    ((96, 80), 3, 3, 2, 1, 0, True),
    ((64, 64), 2, 4, 3, 2, 0, False),
    ((70, 90), 2, 2, 2, 1, 8, True),
    ((48, 48), 1, 3, 2, 0, 0, True),
])
def test_adjoint_matches_oracle_autograd(ofv, shape, levels, kr, it, nr, bits, with_init):
    say("adjoint", shape, levels, kr, it, nr, bits, with_init)
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
    g0, g1, gi = ofv.compute_flow_backward(f0, f1, prm, g_up.float().cuda().contiguous(), flow_init=gi_in,
                                           bit_depth=bits or None)
    torch.cuda.synchronize()
    for name, got, ref in (("frame0", g0, r0), ("frame1", g1, r1), ("flow_init", gi, ri)):
        if ref is None:
            assert got is None
            continue
        rel, cos = _metrics(got, ref)
        say(f"  {name}: rel-L2 {rel:.2e} cosine {cos:.7f}")
        assert rel <= 1e-3 and cos >= 0.9999


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
