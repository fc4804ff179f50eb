"""C-ABI checks that need no GPU: exports, struct layout, argument validation.

A handle created with device -1 owns no device resources; its compute calls
run every host-side check and then return OFV_ERR_UNSUPPORTED, so each
validation branch can be exercised here.
"""
import ctypes
import os
import re
import subprocess
from ctypes import byref, c_int64, c_size_t, c_void_p

import pytest

from paper_2509_25924_amd import _build, _lib
from paper_2509_25924_amd._lib import OfvImage, OfvParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("ofv.h", "ofv_stages.h")]


@pytest.fixture(scope="module")
def lib():
    if not _build.built():
        _build.build()
    return _lib.load()


def _declared_functions():
    names = []
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(ofv_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_every_declared_function_is_exported(lib):
    declared = _declared_functions()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ofv_\w+)", out))
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    # and the binding declares each of them
    assert set(declared) <= set(_lib.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ofv.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ofv_image), offsetof(ofv_image, pitch),'
        ' offsetof(ofv_image, bit_depth), sizeof(ofv_params), offsetof(ofv_params, norm_eps),'
        ' offsetof(ofv_params, flags)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    assert vals == [ctypes.sizeof(OfvImage), OfvImage.pitch.offset, OfvImage.bit_depth.offset,
                    ctypes.sizeof(OfvParams), OfvParams.norm_eps.offset, OfvParams.flags.offset]


def test_default_params(lib):
    p = OfvParams()
    lib.ofv_default_params(byref(p))
    assert (p.num_levels, p.kernel_radius, p.iterations, p.norm_radius) == (3, 4, 3, 1)
    assert abs(p.norm_eps - 1e-4) < 1e-10 and abs(p.reg_rel - 1e-3) < 1e-9 and p.storage == 0 and p.flags == 0
    lib.ofv_default_params(None)


def test_status_strings(lib):
    for s in range(-5, 1):
        assert lib.ofv_status_string(s)
    assert lib.ofv_status_string(-99) == b"unknown status"


@pytest.fixture
def vhandle(lib):
    h = c_void_p()
    assert lib.ofv_create(byref(h), -1, 256, 128, 2, None) == _lib.OFV_OK
    yield h
    assert lib.ofv_destroy(h) == _lib.OFV_OK


def _img(ptr=0x100000, w=64, h=32, pitch=None, typ=_lib.PIX_U8, bits=8):
    return OfvImage(ptr, w, h, pitch if pitch is not None else w, typ, bits)


def _params(**kw):
    p = OfvParams()
    _lib.load().ofv_default_params(byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


OUT = 0x90000000


def _call(lib, h, i0, i1, p, out=OUT):
    return lib.ofv_compute_flow(h, byref(i0), byref(i1), byref(p), c_void_p(out))


def test_create_rejects_bad_arguments(lib):
    h = c_void_p()
    assert lib.ofv_create(None, -1, 8, 8, 1, None) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_create(byref(h), -1, 0, 8, 1, None) == _lib.OFV_ERR_INVALID_ARG
    assert h.value is None
    assert b"max sizes" in lib.ofv_last_error(None)
    assert lib.ofv_create(byref(h), -1, 8, 8, 0, None) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_create(byref(h), -2, 8, 8, 1, None) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_destroy(None) == _lib.OFV_OK


def test_workspace_size_reported(lib, vhandle):
    n = c_size_t()
    assert lib.ofv_workspace_bytes(vhandle, byref(n)) == _lib.OFV_OK
    # 2 pairs x (2 pyramid slabs of ~4/3 x 256x128 floats + 2 flow buffers of 2 x 256x128 floats)
    assert 2 * (2 * 4 * 256 * 128 * 4 // 3 + 2 * 2 * 256 * 128 * 4) <= n.value < 2 * 1_000_000
    assert lib.ofv_workspace_bytes(vhandle, None) == _lib.OFV_ERR_INVALID_ARG


def test_valid_call_reaches_the_device_step(lib, vhandle):
    assert _call(lib, vhandle, _img(), _img(0x200000), _params()) == _lib.OFV_ERR_UNSUPPORTED
    assert b"validation-only" in lib.ofv_last_error(vhandle)


@pytest.mark.parametrize("mut,status,msg", [
    (lambda i0, i1, p: setattr(i0, "data", None), _lib.OFV_ERR_INVALID_ARG, b"data is NULL"),
    (lambda i0, i1, p: setattr(i0, "width", 0), _lib.OFV_ERR_INVALID_ARG, b"size"),
    (lambda i0, i1, p: setattr(i1, "height", -3), _lib.OFV_ERR_INVALID_ARG, b"size"),
    (lambda i0, i1, p: setattr(i0, "pitch", 10), _lib.OFV_ERR_INVALID_ARG, b"pitch"),
    (lambda i0, i1, p: setattr(i0, "bit_depth", 9), _lib.OFV_ERR_INVALID_ARG, b"bit_depth"),
    (lambda i0, i1, p: (setattr(i0, "type", _lib.PIX_U16), setattr(i0, "bit_depth", 17)), _lib.OFV_ERR_INVALID_ARG,
     b"bit_depth"),
    (lambda i0, i1, p: setattr(i0, "type", 7), _lib.OFV_ERR_INVALID_ARG, b"pixel type"),
    (lambda i0, i1, p: setattr(i1, "width", 63), _lib.OFV_ERR_INVALID_ARG, b"sizes differ"),
    (lambda i0, i1, p: setattr(p, "num_levels", 0), _lib.OFV_ERR_INVALID_ARG, b"num_levels"),
    (lambda i0, i1, p: setattr(p, "num_levels", 17), _lib.OFV_ERR_INVALID_ARG, b"num_levels"),
    (lambda i0, i1, p: setattr(p, "kernel_radius", 0), _lib.OFV_ERR_INVALID_ARG, b"kernel_radius"),
    (lambda i0, i1, p: setattr(p, "kernel_radius", 13), _lib.OFV_ERR_UNSUPPORTED, b"kernel_radius"),
    (lambda i0, i1, p: setattr(p, "iterations", 0), _lib.OFV_ERR_INVALID_ARG, b"iterations"),
    (lambda i0, i1, p: setattr(p, "norm_radius", -1), _lib.OFV_ERR_INVALID_ARG, b"norm_radius"),
    (lambda i0, i1, p: setattr(p, "norm_radius", 17), _lib.OFV_ERR_INVALID_ARG, b"norm_radius"),
    (lambda i0, i1, p: setattr(p, "norm_eps", float("nan")), _lib.OFV_ERR_INVALID_ARG, b"norm_eps"),
    (lambda i0, i1, p: setattr(p, "reg_rel", -1.0), _lib.OFV_ERR_INVALID_ARG, b"reg_rel"),
    (lambda i0, i1, p: setattr(p, "reg_abs", float("inf")), _lib.OFV_ERR_INVALID_ARG, b"reg_abs"),
    (lambda i0, i1, p: setattr(p, "storage", 3), _lib.OFV_ERR_INVALID_ARG, b"storage"),
    (lambda i0, i1, p: setattr(p, "flags", 64), _lib.OFV_ERR_INVALID_ARG, b"flags"),
    (lambda i0, i1, p: (setattr(i0, "width", 257), setattr(i1, "width", 257), setattr(i0, "pitch", 257),
                        setattr(i1, "pitch", 257)), _lib.OFV_ERR_CAPACITY, b"exceeds"),
    (lambda i0, i1, p: (setattr(i0, "height", 129), setattr(i1, "height", 129)), _lib.OFV_ERR_CAPACITY, b"exceeds"),
])
def test_compute_rejects_bad_arguments(lib, vhandle, mut, status, msg):
    i0, i1, p = _img(), _img(0x200000), _params()
    mut(i0, i1, p)
    assert _call(lib, vhandle, i0, i1, p) == status
    assert msg in lib.ofv_last_error(vhandle)


def test_null_arguments(lib, vhandle):
    i0, i1, p = _img(), _img(0x200000), _params()
    assert lib.ofv_compute_flow(None, byref(i0), byref(i1), byref(p), c_void_p(OUT)) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_compute_flow(vhandle, None, byref(i1), byref(p), c_void_p(OUT)) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_compute_flow(vhandle, byref(i0), byref(i1), None, c_void_p(OUT)) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_compute_flow(vhandle, byref(i0), byref(i1), byref(p), None) == _lib.OFV_ERR_INVALID_ARG


def test_output_aliasing_is_rejected(lib, vhandle):
    i0, i1, p = _img(), _img(0x200000), _params()
    # flow_out overlapping either frame
    assert _call(lib, vhandle, i0, i1, p, out=0x100000 + 100) == _lib.OFV_ERR_INVALID_ARG
    assert b"overlaps frame0" in lib.ofv_last_error(vhandle)
    assert _call(lib, vhandle, i0, i1, p, out=0x200000 - 8) == _lib.OFV_ERR_INVALID_ARG
    # flow_init may equal flow_out but not partially overlap it
    assert lib.ofv_compute_flow_ex(vhandle, byref(i0), byref(i1), byref(p), c_void_p(OUT),
                                   c_void_p(OUT)) == _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_compute_flow_ex(vhandle, byref(i0), byref(i1), byref(p), c_void_p(OUT + 4),
                                   c_void_p(OUT)) == _lib.OFV_ERR_INVALID_ARG


def test_batch_validation(lib, vhandle):
    n = 3
    a0 = (OfvImage * n)(*[_img(0x100000 * (k + 1)) for k in range(n)])
    a1 = (OfvImage * n)(*[_img(0x1000000 + 0x100000 * k) for k in range(n)])
    outs = (c_void_p * n)(*[OUT + 0x100000 * k for k in range(n)])
    p = _params()
    assert lib.ofv_compute_flow_batch(vhandle, n, a0, a1, byref(p), None, outs) == _lib.OFV_ERR_CAPACITY
    assert lib.ofv_compute_flow_batch(vhandle, 0, a0, a1, byref(p), None, outs) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_compute_flow_batch(vhandle, 2, a0, a1, byref(p), None, outs) == _lib.OFV_ERR_UNSUPPORTED
    outs2 = (c_void_p * 2)(OUT, OUT + 64)
    assert lib.ofv_compute_flow_batch(vhandle, 2, a0, a1, byref(p), None, outs2) == _lib.OFV_ERR_INVALID_ARG
    assert b"overlaps flow_out" in lib.ofv_last_error(vhandle)


def test_stage_validation(lib, vhandle):
    img = _img()
    assert lib.ofv_stage_normalize(vhandle, byref(img), 2, 1e-4, 0, c_void_p(OUT), 64) == _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_stage_normalize(vhandle, byref(img), 2, 1e-4, 0, c_void_p(OUT), 32) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stage_normalize(vhandle, byref(img), 99, 1e-4, 0, c_void_p(OUT), 64) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stage_reduce(vhandle, 0, c_void_p(0x1000), 10, 10, 9, c_void_p(OUT), 5) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stage_reduce(vhandle, 0, c_void_p(0x1000), 10, 10, 10, c_void_p(OUT), 5) == _lib.OFV_ERR_UNSUPPORTED
    outs = (c_void_p * 3)(OUT, OUT + 0x10000, OUT + 0x20000)
    pitches = (c_int64 * 3)(5, 3, 2)
    for levels in (0, 4):
        assert lib.ofv_stage_pyramid(vhandle, 0, c_void_p(0x1000), 10, 10, 10, levels, outs, pitches) == \
            _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stage_pyramid(vhandle, 0, c_void_p(0x1000), 10, 10, 10, 3, None, pitches) == _lib.OFV_ERR_INVALID_ARG
    pitches[1] = 2
    assert lib.ofv_stage_pyramid(vhandle, 0, c_void_p(0x1000), 10, 10, 10, 3, outs, pitches) == _lib.OFV_ERR_INVALID_ARG
    pitches[1] = 3
    assert lib.ofv_stage_pyramid(vhandle, 3, c_void_p(0x1000), 10, 10, 10, 3, outs, pitches) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stage_pyramid(vhandle, 0, c_void_p(0x1000), 10, 10, 10, 3, outs, pitches) == \
        _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_stage_upsample(vhandle, c_void_p(0x1000), 5, 5, 5, c_void_p(OUT), 10, 10, 10) == \
        _lib.OFV_ERR_UNSUPPORTED
    args = [vhandle, 0, c_void_p(0x1000), c_void_p(0x2000), 16, 16, 16, _lib.FLOW_IN_DIRECT, c_void_p(OUT), 16, 16,
            16, c_void_p(OUT + 16), 16, 4, 1e-3, 1e-9]
    assert lib.ofv_stage_gn_iteration(*args) == _lib.OFV_ERR_INVALID_ARG      # output overlaps input
    args[12] = c_void_p(OUT + 1 << 20)
    assert lib.ofv_stage_gn_iteration(*args) == _lib.OFV_ERR_UNSUPPORTED
    args[14] = 13
    assert lib.ofv_stage_gn_iteration(*args) == _lib.OFV_ERR_UNSUPPORTED
    args[14] = 4
    args[7] = 5
    assert lib.ofv_stage_gn_iteration(*args) == _lib.OFV_ERR_INVALID_ARG


def test_fault_injection_reports_device_error(lib, vhandle, monkeypatch):
    monkeypatch.setenv("OFV_FAULT_INJECT", "launch")
    assert _call(lib, vhandle, _img(), _img(0x200000), _params()) == _lib.OFV_ERR_DEVICE
    assert b"injected" in lib.ofv_last_error(vhandle)
    monkeypatch.setenv("OFV_FAULT_INJECT", "alloc")
    h = c_void_p()
    assert lib.ofv_create(byref(h), 0, 64, 64, 1, None) == _lib.OFV_ERR_OUT_OF_MEMORY
    assert h.value is None


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load(str(tmp_path / "nope.so"))


def test_derived_validation(lib, vhandle):
    p = _lib.OfvDerivedParams()
    lib.ofv_default_derived_params(byref(p))
    assert (p.dx, p.dz, p.dt, p.streamwise_sign) == (1.0, 1.0, 1.0, 1)
    flow, vort, area = c_void_p(0x100000), c_void_p(0x900000), c_void_p(0xA00000)
    args = [vhandle, flow, 64, 32, 64, None, 0, byref(p), vort, 64, None, 0, None, area]
    assert lib.ofv_derived(*args) == _lib.OFV_ERR_UNSUPPORTED             # valid, validation-only handle
    bad = list(args); bad[1] = None
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    bad = list(args); bad[4] = 63
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    bad = list(args); bad[9] = 10
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    bad = list(args); bad[5] = c_void_p(0x800000)                           # mask with pitch 0
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    bad = list(args); bad[8] = c_void_p(0x100000 + 64 * 4)                  # vorticity inside the flow
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    assert b"overlaps" in lib.ofv_last_error(vhandle)
    bad = list(args); bad[11] = 3                                           # probes without arrays
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    bad = list(args); bad[11] = (1 << 20) + 1
    assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG
    for field, val in (("dx", 0.0), ("dz", -1.0), ("dt", float("inf")), ("streamwise_sign", 2)):
        q = _lib.OfvDerivedParams(p.dx, p.dz, p.dt, p.streamwise_sign)
        setattr(q, field, val)
        bad = list(args); bad[7] = byref(q)
        assert lib.ofv_derived(*bad) == _lib.OFV_ERR_INVALID_ARG, field
    none = [vhandle, flow, 64, 32, 64, None, 0, byref(p), None, 0, None, 0, None, None]
    assert lib.ofv_derived(*none) == _lib.OFV_OK                            # nothing requested


def test_stream_validation(lib, vhandle):
    img = _img()
    p = _params()
    produced = ctypes.c_int(7)
    assert lib.ofv_stream_push(vhandle, byref(img), byref(p), None, c_void_p(OUT), None) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stream_push(vhandle, None, byref(p), None, c_void_p(OUT), byref(produced)) == \
        _lib.OFV_ERR_INVALID_ARG
    bad = _params(num_levels=0)
    assert lib.ofv_stream_push(vhandle, byref(img), byref(bad), None, c_void_p(OUT), byref(produced)) == \
        _lib.OFV_ERR_INVALID_ARG
    assert produced.value == 0
    assert lib.ofv_stream_push(vhandle, byref(img), byref(p), None, None, byref(produced)) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_stream_push(vhandle, byref(img), byref(p), None, c_void_p(OUT), byref(produced)) == \
        _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_stream_reset(vhandle) == _lib.OFV_OK
    assert lib.ofv_stream_reset(None) == _lib.OFV_ERR_INVALID_ARG


def test_estimator_flags(lib, vhandle):
    img0, img1 = _img(), _img(0x200000)
    p = _params(flags=_lib.FLAG_FORWARD_ADDITIVE)
    assert lib.ofv_compute_flow(vhandle, byref(img0), byref(img1), byref(p), c_void_p(OUT)) == \
        _lib.OFV_ERR_UNSUPPORTED                                        # valid, validation-only handle
    for ok in (_lib.FLAG_INCREMENT_UPDATE, _lib.FLAG_NO_FP64_FALLBACK, _lib.FLAG_STORE_ALL,
               _lib.FLAG_FORWARD_ADDITIVE | _lib.FLAG_INCREMENT_UPDATE | _lib.FLAG_NO_FP64_FALLBACK):
        q = _params(flags=ok)
        assert lib.ofv_compute_flow(vhandle, byref(img0), byref(img1), byref(q), c_void_p(OUT)) == \
            _lib.OFV_ERR_UNSUPPORTED
    bad = _params(flags=64)
    assert lib.ofv_compute_flow(vhandle, byref(img0), byref(img1), byref(bad), c_void_p(OUT)) == \
        _lib.OFV_ERR_INVALID_ARG
    for est in (_lib.FLAG_FORWARD_ADDITIVE, _lib.FLAG_INCREMENT_UPDATE):
        q = _params(flags=est)
        assert lib.ofv_compute_flow_backward(vhandle, byref(img0), byref(img1), byref(q), None, c_void_p(OUT),
                                             c_void_p(OUT + (1 << 20)), None, None) == _lib.OFV_ERR_UNSUPPORTED
        assert b"symmetric" in lib.ofv_last_error(vhandle)


def test_static_entry_point_validation(lib, monkeypatch):
    """ofv_compute_flow_static checks everything on the host before touching a device: bad
    arguments, and pairs whose workspace exceeds the static scratch array (OFV_ERR_CAPACITY)."""
    def call(i0, i1, p, out=OUT):
        return lib.ofv_compute_flow_static(byref(i0), byref(i1), byref(p), c_void_p(out), None)

    assert lib.ofv_compute_flow_static(None, byref(_img()), byref(_params()), c_void_p(OUT), None) == \
        _lib.OFV_ERR_INVALID_ARG
    assert b"frame0 is NULL" in lib.ofv_last_error(None)
    assert call(_img(), _img(0x200000), _params(kernel_radius=0)) == _lib.OFV_ERR_INVALID_ARG
    assert b"kernel_radius" in lib.ofv_last_error(None)
    assert call(_img(), _img(0x200000, w=65), _params()) == _lib.OFV_ERR_INVALID_ARG
    assert b"sizes differ" in lib.ofv_last_error(None)
    assert call(_img(), _img(0x200000), _params(), out=0) == _lib.OFV_ERR_INVALID_ARG
    big0 = _img(0x100000, w=2048, h=1024)
    big1 = _img(0x40000000, w=2048, h=1024)
    assert call(big0, big1, _params(), out=0x80000000) == _lib.OFV_ERR_CAPACITY
    assert b"static scratch" in lib.ofv_last_error(None)
    fit0 = _img(0x100000, w=1280, h=1024)
    fit1 = _img(0x40000000, w=1280, h=1024)
    monkeypatch.setenv("OFV_FAULT_INJECT", "launch")
    assert call(fit0, fit1, _params(), out=0x80000000) == _lib.OFV_ERR_DEVICE
    assert b"injected" in lib.ofv_last_error(None)


def test_sync_fault_injection_on_destroy(lib, monkeypatch):
    """OFV_FAULT_INJECT=sync: the synchronisation in ofv_destroy reports a device error (the handle is
    released all the same); without the injection the same call succeeds."""
    h = c_void_p()
    assert lib.ofv_create(byref(h), -1, 64, 64, 1, None) == _lib.OFV_OK
    monkeypatch.setenv("OFV_FAULT_INJECT", "sync")
    assert lib.ofv_destroy(h) == _lib.OFV_ERR_DEVICE
    monkeypatch.setenv("OFV_FAULT_INJECT", "alloc,sync")
    h2 = c_void_p()
    assert lib.ofv_create(byref(h2), -1, 64, 64, 1, None) == _lib.OFV_OK   # validation-only: nothing allocated
    assert lib.ofv_destroy(h2) == _lib.OFV_ERR_DEVICE
    monkeypatch.delenv("OFV_FAULT_INJECT")
    h3 = c_void_p()
    assert lib.ofv_create(byref(h3), -1, 64, 64, 1, None) == _lib.OFV_OK
    assert lib.ofv_destroy(h3) == _lib.OFV_OK


def test_backward_workspace_bytes(lib, vhandle):
    """Reservation sizes (256 x 128 handle, pitches equal widths at these levels): the store-all
    record adds 8 planes per level and iteration plus the first iteration's input field per level,
    and the workspace scales with the number of pairs."""
    def nbytes(L, it, pairs, mode):
        out = ctypes.c_size_t()
        assert lib.ofv_backward_workspace_bytes(vhandle, L, it, pairs, mode, byref(out)) == _lib.OFV_OK
        return out.value
    for L, it in ((1, 1), (3, 3), (2, 5)):
        rc = nbytes(L, it, 1, 0)
        sa = nbytes(L, it, 1, _lib.BACKWARD_STORE_ALL)
        planes = sum((256 >> l) * (128 >> l) for l in range(L))
        assert sa - rc == 4 * (8 * it + 2) * planes
        assert nbytes(L, it, 2, 0) == 2 * rc and nbytes(L, it, 2, _lib.BACKWARD_STORE_ALL) == 2 * sa
        # the saved output fields and the 15 level-0 scratch planes are in there
        assert rc >= 4 * (2 * it * planes + 15 * 256 * 128)
    out = ctypes.c_size_t()
    for args in ((0, 3, 1, 0), (3, 0, 1, 0), (3, 3, 0, 0), (3, 3, 3, 0), (3, 3, 1, 2)):
        assert lib.ofv_backward_workspace_bytes(vhandle, *args, byref(out)) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_backward_workspace_bytes(vhandle, 3, 3, 1, 0, None) == _lib.OFV_ERR_INVALID_ARG
    assert lib.ofv_backward_workspace_bytes(None, 3, 3, 1, 0, byref(out)) == _lib.OFV_ERR_INVALID_ARG
    # a validation-only handle cannot allocate
    assert lib.ofv_reserve_backward_ex(vhandle, 3, 3, 1, 0) == _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_reserve_backward_ex(vhandle, 3, 3, 3, 0) == _lib.OFV_ERR_INVALID_ARG   # above max_batch


def test_backward_batch_validation(lib, vhandle):
    """ofv_compute_flow_backward_batch checks the batch on the host: sizes, NULL arrays, overlaps
    between any output and any input or output of the batch, and the reservation."""
    n = 2
    i0 = (OfvImage * n)(_img(0x100000), _img(0x300000))
    i1 = (OfvImage * n)(_img(0x200000), _img(0x400000))
    p = _params()
    gflow = (c_void_p * n)(0x1000000, 0x1100000)
    g0 = (c_void_p * n)(0x2000000, 0x2100000)

    def call(nn=n, a0=i0, a1=i1, pp=p, init=None, gf=gflow, o0=g0, o1=None, oi=None):
        return lib.ofv_compute_flow_backward_batch(vhandle, nn, a0, a1, byref(pp), init, gf, o0, o1, oi)
    assert call(nn=0) == _lib.OFV_ERR_INVALID_ARG
    assert call(nn=3) == _lib.OFV_ERR_CAPACITY                    # max_batch 2
    assert call(gf=None) == _lib.OFV_ERR_INVALID_ARG
    assert call(gf=(c_void_p * n)(0x1000000, None)) == _lib.OFV_ERR_INVALID_ARG
    # grad_frame0 of pair 1 overlaps frame1 of pair 0
    assert call(o0=(c_void_p * n)(0x2000000, 0x200000)) == _lib.OFV_ERR_INVALID_ARG
    assert b"overlaps" in lib.ofv_last_error(vhandle)
    # two outputs of different pairs overlap
    assert call(o1=(c_void_p * n)(0x2100000, None)) == _lib.OFV_ERR_INVALID_ARG
    # grad_flow_init without flow_init
    assert call(oi=(c_void_p * n)(None, 0x3000000)) == _lib.OFV_ERR_INVALID_ARG
    assert b"flow_init" in lib.ofv_last_error(vhandle)
    p16 = _params(storage=_lib.STORE["f16"])
    assert call(pp=p16) == _lib.OFV_ERR_UNSUPPORTED
    big = (OfvImage * n)(_img(0x100000), _img(0x300000, w=512))
    assert call(a0=big, a1=(OfvImage * n)(_img(0x200000), _img(0x400000, w=512))) == _lib.OFV_ERR_CAPACITY
    # valid batch, no reservation on this handle
    assert call() == _lib.OFV_ERR_CAPACITY
    assert b"ofv_reserve_backward_ex" in lib.ofv_last_error(vhandle)
    assert call(pp=_params(flags=_lib.FLAG_STORE_ALL)) == _lib.OFV_ERR_CAPACITY


def test_save_iterates_validation(lib, vhandle):
    """A forward that keeps its iterates needs the adjoint's estimator and storage and a reservation;
    the static and streaming entry points and the autotuner reject it."""
    img0, img1 = _img(), _img(0x200000)
    p = _params(flags=_lib.FLAG_SAVE_ITERATES)
    assert lib.ofv_compute_flow(vhandle, byref(img0), byref(img1), byref(p), c_void_p(OUT)) == _lib.OFV_ERR_CAPACITY
    assert b"ofv_reserve_backward_ex" in lib.ofv_last_error(vhandle)
    for bad in (_params(flags=_lib.FLAG_SAVE_ITERATES | _lib.FLAG_FORWARD_ADDITIVE),
                _params(flags=_lib.FLAG_SAVE_ITERATES, storage=_lib.STORE["bf16"])):
        assert lib.ofv_compute_flow(vhandle, byref(img0), byref(img1), byref(bad), c_void_p(OUT)) == \
            _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_compute_flow_static(byref(img0), byref(img1), byref(p), c_void_p(OUT), None) == \
        _lib.OFV_ERR_UNSUPPORTED
    produced = ctypes.c_int()
    assert lib.ofv_stream_push(vhandle, byref(img0), byref(p), None, c_void_p(OUT), byref(produced)) == \
        _lib.OFV_ERR_UNSUPPORTED
    assert lib.ofv_autotune(vhandle, byref(img0), byref(img1), byref(p), c_void_p(OUT), 1) == _lib.OFV_ERR_UNSUPPORTED
    # the backward accepts the saved-forward flag (and still needs its reservation)
    q = _params(flags=_lib.FLAG_SAVED_FORWARD)
    assert lib.ofv_compute_flow_backward(vhandle, byref(img0), byref(img1), byref(q), None, c_void_p(OUT),
                                         c_void_p(OUT + (1 << 20)), None, None) == _lib.OFV_ERR_CAPACITY


def test_tuning_import_validation(lib, vhandle):
    """Tile heights 4..1024 for every decomposition, and 0 (sized from the occupancy at every launch) for the
    band only; a malformed entry merges nothing."""
    for ok in (b"10 0 1 5120 4096 1 11 0\n", b"10 0 1 5120 4096 1 11 128\n", b"5 0 1 1024 1024 1 7 64\n"):
        assert lib.ofv_tuning_import(vhandle, ok) == _lib.OFV_OK, ok
    for bad in (b"10 0 1 5120 4096 1 11 2\n", b"5 0 1 1024 1024 1 7 0\n", b"10 0 1 2560 2048 1 12 0\n",
                b"10 0 1 2560 2048 1 11 2048\n", b"10 0 1 2560 2048 1 11\n"):
        assert lib.ofv_tuning_import(vhandle, b"4 0 1 256 256 1 4 16\n" + bad) == _lib.OFV_ERR_INVALID_ARG, bad
    need = c_size_t(0)
    assert lib.ofv_tuning_export(vhandle, None, 0, byref(need)) == _lib.OFV_OK
    buf = ctypes.create_string_buffer(need.value)
    assert lib.ofv_tuning_export(vhandle, buf, need.value, byref(need)) == _lib.OFV_OK
    lines = set(buf.value.decode().split("\n"))
    assert "10 0 1 5120 4096 1 11 128" in lines and "5 0 1 1024 1024 1 7 64" in lines
    assert not any(l.startswith("4 0 1 256 256") for l in lines)        # the rejected texts merged nothing
