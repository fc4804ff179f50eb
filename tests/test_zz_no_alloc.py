"""ofv_compute_flow_static, the entry point that allocates nothing: through the
C ABI it must give exactly what ofv_compute_flow gives with the default
work decomposition (same kernels, its workspace a static device array of the
library instead of a handle's), on calls in a row of decreasing size, and
reject pairs too large for that array before enqueuing anything."""
import sys
from ctypes import byref, c_void_p

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


def _static_call(ofv, f0, f1, prm, bits, out):
    from paper_2509_25924_amd import _lib
    from paper_2509_25924_amd.api import image_desc, params_struct
    lib = ofv.load()
    i0, i1 = image_desc(f0, bits), image_desc(f1, bits)
    p = params_struct(prm)
    return lib.ofv_compute_flow_static(byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr()),
                                       c_void_p(torch.cuda.current_stream().cuda_stream)), _lib


def test_static_entry_point_equals_handle_call(ofv):
    cases = [((384, 512), synth.Translation(1.37, -0.62), 12, {"num_levels": 4, "kernel_radius": 5,
                                                                "iterations": 4, "norm_radius": 1}),
             ((150, 200), synth.Translation(-0.8, 0.45), 8, {"num_levels": 3, "kernel_radius": 4,
                                                             "iterations": 3, "norm_radius": 1})]
    for k, ((h, w), flow, bits, prm) in enumerate(cases):
        say(f"static entry point, call {k}: {w}x{h}, {bits}-bit, {prm}")
        pair = synth.make_pair(h, w, flow, fwhm=2.5, ppp=0.1, seed=700 + k, bit_depth=bits,
                               noise=2 if bits == 8 else 40.95)
        f0 = torch.from_numpy(pair.frame0).cuda()
        f1 = torch.from_numpy(pair.frame1).cuda()
        out = torch.full((2, h, w), float("nan"), dtype=torch.float32, device="cuda")
        st, _lib = _static_call(ofv, f0, f1, prm, bits, out)
        assert st == _lib.OFV_OK, ofv.load().ofv_last_error(None)
        handle = ofv.Handle(w, h, 1)
        handle.set_gn_variant("auto")
        want = ofv.compute_flow(f0, f1, prm, bit_depth=bits, handle=handle)
        torch.cuda.synchronize()
        assert torch.equal(out, want), float((out - want).abs().max())
        ref = oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=bits)
        err = float(np.max(np.abs(out.cpu().double().numpy() - ref.numpy())))
        say(f"  bitwise equal to the handle call; max |dV| vs FP64 oracle {err:.2e} px")
        assert err <= 1e-3
        handle.close()


def test_static_entry_point_rejects_oversize(ofv):
    h, w = 1024, 2048
    f0 = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
    out = torch.full((2, h, w), 7.0, dtype=torch.float32, device="cuda")
    st, _lib = _static_call(ofv, f0, f0.clone(), {"num_levels": 3, "kernel_radius": 4, "iterations": 3,
                                                  "norm_radius": 1}, 8, out)
    torch.cuda.synchronize()
    assert st == _lib.OFV_ERR_CAPACITY
    assert b"static scratch" in ofv.load().ofv_last_error(None)
    assert bool((out == 7.0).all())
