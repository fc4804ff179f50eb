"""Forced failures on a device handle (OFV_FAULT_INJECT): every call returns a
clean status, a failing compute call writes nothing, and the handle keeps
working once the injection is lifted.  All conditions are forced from the
host; no kernel is made to fault."""
import sys
from ctypes import byref, c_void_p

import pytest
import torch

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


def test_injected_launch_failure_writes_nothing(ofv, monkeypatch):
    say("fault injection: launch")
    from paper_2509_25924_amd import _lib
    pair, prm = synth.config_rankine_256(size=128)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    h = ofv.Handle(128, 128, 1)
    out = torch.full((2, 128, 128), 3.25, dtype=torch.float32, device="cuda")
    monkeypatch.setenv("OFV_FAULT_INJECT", "launch")
    with pytest.raises(ofv.OfvError) as e:
        ofv.compute_flow(f0, f1, prm, bit_depth=8, out=out, handle=h)
    assert e.value.status == _lib.OFV_ERR_DEVICE
    with pytest.raises(ofv.OfvError):
        ofv.compute_flow_static(f0, f1, prm, bit_depth=8, out=out)
    torch.cuda.synchronize()
    assert bool((out == 3.25).all())
    monkeypatch.delenv("OFV_FAULT_INJECT")
    ofv.compute_flow(f0, f1, prm, bit_depth=8, out=out, handle=h)   # the handle still works
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all()) and not bool((out == 3.25).all())
    h.close()


def test_injected_sync_failure(ofv, monkeypatch):
    say("fault injection: sync")
    from paper_2509_25924_amd import _lib
    pair, prm = synth.config_rankine_256(size=128)
    f0 = torch.from_numpy(pair.frame0).cuda()
    f1 = torch.from_numpy(pair.frame1).cuda()
    lib = ofv.load()
    h = c_void_p()
    assert lib.ofv_create(byref(h), torch.cuda.current_device(), 128, 128, 1,
                          c_void_p(torch.cuda.current_stream().cuda_stream)) == _lib.OFV_OK
    from paper_2509_25924_amd.api import image_desc, params_struct
    i0, i1, p = image_desc(f0, 8), image_desc(f1, 8), params_struct(prm)
    out = torch.empty((2, 128, 128), dtype=torch.float32, device="cuda")
    monkeypatch.setenv("OFV_FAULT_INJECT", "sync")
    # the autotuner synchronises after each candidate: it stops with a device error
    assert lib.ofv_autotune(h, byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr()), 1) == _lib.OFV_ERR_DEVICE
    assert b"synchronisation" in lib.ofv_last_error(h)
    # compute calls do not synchronise: unaffected
    assert lib.ofv_compute_flow(h, byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr())) == _lib.OFV_OK
    torch.cuda.synchronize()
    # destroy reports the failed synchronisation and still releases the handle
    assert lib.ofv_destroy(h) == _lib.OFV_ERR_DEVICE
    monkeypatch.delenv("OFV_FAULT_INJECT")


def test_injected_alloc_failure(ofv, monkeypatch):
    say("fault injection: alloc")
    from paper_2509_25924_amd import _lib
    lib = ofv.load()
    monkeypatch.setenv("OFV_FAULT_INJECT", "alloc")
    h = c_void_p()
    assert lib.ofv_create(byref(h), torch.cuda.current_device(), 256, 256, 1, None) == _lib.OFV_ERR_OUT_OF_MEMORY
    assert h.value is None
    monkeypatch.delenv("OFV_FAULT_INJECT")
    hd = ofv.Handle(64, 64, 1)
    monkeypatch.setenv("OFV_FAULT_INJECT", "alloc")
    with pytest.raises(ofv.OfvError) as e:
        hd.reserve_backward(2, 2)
    assert e.value.status == _lib.OFV_ERR_OUT_OF_MEMORY
    monkeypatch.delenv("OFV_FAULT_INJECT")
    hd.reserve_backward(2, 2)
    hd.close()
