"""Parity of the live derived quantities (vorticity, recirculation area of
Eq. RA, velocity probes) computed by the HIP kernel through the C ABI with
the FP64 oracle on the same float32 field.  The pixel count behind the area
is integer work and must match exactly; vorticity and probes are float32
arithmetic on float32 inputs and must agree to a few roundings."""
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


def _check(ofv, flow, mask=None, dx=1.0, dz=1.0, dt=1.0, sign=1, probes=None, handle=None):
    """Runs the kernel and the oracle on the same float32 field and compares."""
    dx, dz, dt = (float(np.float32(q)) for q in (dx, dz, dt))   # the C ABI takes them as float32
    f = torch.as_tensor(flow, dtype=torch.float32)
    dev = f.cuda()
    dmask = torch.as_tensor(mask).cuda() if mask is not None else None
    dpr = torch.as_tensor(probes, dtype=torch.float32).cuda() if probes is not None else None
    got = ofv.derived(dev, dmask, dx, dz, dt, sign, dpr, handle=handle)
    torch.cuda.synchronize()
    u, v = f[0].double(), f[1].double()
    om = oracle.vorticity(u, v, dx, dz, dt, mask=mask)
    scale = (dz / dx + dx / dz) / dt * max(float(f.abs().max()), 1e-30)
    err = torch.max(torch.abs(got["vorticity"].cpu().double() - om)).item()
    assert err <= 4e-7 * scale, (err, scale)
    area, n = oracle.recirculation_area(u, dx, dz, mask=mask, sign=sign)
    assert got["area"].item() == area, (got["area"].item(), area, n)
    if probes is not None:
        pr = oracle.probes(u, v, torch.as_tensor(probes, dtype=torch.float64), dx, dz, dt)
        sc = max(dx, dz) / dt * max(float(f.abs().max()), 1e-30)
        assert torch.max(torch.abs(got["probes"].cpu().double() - pr)).item() <= 4e-7 * sc
    return got


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (7, 1), (2, 2), (3, 5), (16, 64), (17, 65), (65, 130),
                                   (257, 255), (1000, 1366)])
def test_random_fields_with_mask(ofv, shape):
    say("derived", shape)
    rng = np.random.default_rng(sum(shape))
    flow = rng.normal(0, 2, (2,) + shape).astype(np.float32)
    flow[0][rng.random(shape) < 0.05] = 0.0          # exact zeros are not recirculating
    mask = (rng.random(shape) > 0.2).astype(np.uint8)
    pts = np.stack([rng.uniform(-3, shape[1] + 3, 300), rng.uniform(-3, shape[0] + 3, 300)], 1).astype(np.float32)
    _check(ofv, flow, mask, 0.5, 0.25, 0.01, 1, pts)
    _check(ofv, flow, None, 2.0, 1.0, 1.0, -1, pts[:7])


def test_estimated_wake_field(ofv):
    """The field of the estimator on a cylinder-wake pair, masked inside the cylinder."""
    say("derived on an estimated wake field")
    pair, prm = synth.config_rankine_256(seed=3)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    flow = ofv.compute_flow(f0, f1, prm, bit_depth=8).cpu().numpy()
    h, w = flow.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    mask = (((xx - w / 2) ** 2 + (yy - h / 2) ** 2) > 20 ** 2).astype(np.uint8)
    _check(ofv, flow, mask, 1e-4, 1e-4, 1e-2, 1, np.array([[64.5, 100.25], [200, 30]], np.float32))


def test_repeated_calls_and_graph_replays_keep_the_count(ofv):
    """The per-workgroup counts kept in the handle are rewritten by every call: repeated eager calls
    and several replays of a captured call (with other work in between)
    give the same exact area each time."""
    say("derived counters across calls and graph replays")
    rng = np.random.default_rng(9)
    flow = torch.as_tensor(rng.normal(0, 1, (2, 300, 400)).astype(np.float32)).cuda()
    ref, _ = oracle.recirculation_area(flow[0].cpu().double())
    h = ofv.Handle(16, 16, 1)
    for _ in range(3):
        assert ofv.derived(flow, vorticity=False, handle=h)["area"].item() == ref
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ofv.derived(flow, handle=h)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = ofv.derived(flow, handle=h)
    h.bind_stream()
    for k in range(4):
        g.replay()
        torch.cuda.synchronize()
        assert out["area"].item() == ref, k
        other = ofv.derived(-flow, vorticity=False, handle=h)["area"].item()   # eager work between replays
        torch.cuda.synchronize()
        ref_neg, _ = oracle.recirculation_area(-flow[0].cpu().double())
        assert other == ref_neg
    h.close()


def test_full_size_21mp_field(ofv):
    """5120 x 4096 (the live configuration's full frame): exact count, vorticity checked everywhere."""
    say("derived 5120x4096")
    g = torch.Generator().manual_seed(21)
    flow = (torch.randn((2, 4096, 5120), generator=g) * 3).float()
    mask = (torch.rand((4096, 5120), generator=g) > 0.1).to(torch.uint8).numpy()
    pts = np.array([[0, 0], [5119, 4095], [2560.5, 2048.25], [1024, 2048]], np.float32)
    _check(ofv, flow, mask, 0.1, 0.1, 0.01, 1, pts)


def test_padded_pitches_through_the_c_abi(ofv):
    """Flow, mask and vorticity planes with row pitches above the width, called through the C ABI."""
    from ctypes import byref, c_void_p
    from paper_2509_25924_amd import _lib
    say("derived with padded pitches")
    h, w = 150, 203
    fp, mp, vp = w + 13, w + 5, w + 7
    rng = np.random.default_rng(44)
    flow = rng.normal(0, 1.5, (2, h, w)).astype(np.float32)
    mask = (rng.random((h, w)) > 0.3).astype(np.uint8)
    dflow = torch.full((2, h, fp), float("nan"), device="cuda")
    dflow[:, :, :w] = torch.from_numpy(flow).cuda()
    dmask = torch.zeros((h, mp), dtype=torch.uint8, device="cuda")
    dmask[:, :w] = torch.from_numpy(mask).cuda()
    dvort = torch.full((h, vp), 7.0, device="cuda")
    area = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = ofv.load()
    hd = ofv.Handle(16, 16, 1)
    p = _lib.OfvDerivedParams(0.5, 2.0, 0.25, -1)
    st = lib.ofv_derived(hd.ptr, c_void_p(dflow.data_ptr()), w, h, fp, c_void_p(dmask.data_ptr()), mp, byref(p),
                         c_void_p(dvort.data_ptr()), vp, None, 0, None, c_void_p(area.data_ptr()))
    assert st == 0, lib.ofv_last_error(hd.ptr)
    torch.cuda.synchronize()
    u, v = torch.as_tensor(flow[0]).double(), torch.as_tensor(flow[1]).double()
    om = oracle.vorticity(u, v, 0.5, 2.0, 0.25, mask=mask)
    got = dvort[:, :w].cpu().double()
    assert torch.max(torch.abs(got - om)).item() <= 4e-7 * (2.0 / 0.5 + 0.5 / 2.0) / 0.25 * float(np.abs(flow).max())
    assert torch.all(dvort[:, w:] == 7.0)                 # nothing written past the width
    ref, _ = oracle.recirculation_area(u, 0.5, 2.0, mask=mask, sign=-1)
    assert area.item() == ref
    hd.close()
