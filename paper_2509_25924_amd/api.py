"""Python entry points of the OFV estimator (thin marshalling over libofv.so).

Every step runs in the HIP kernels of libofv.so; this module only turns
torch CUDA tensors into the C structs of include/ofv.h and passes the
current torch stream.  Tensors must live on a ROCm device.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int64, c_size_t, c_void_p
from typing import Dict, List, Optional, Sequence

import torch

from . import _lib
from ._lib import OfvDerivedParams, OfvImage, OfvParams, check, load

_PIX = {torch.uint8: _lib.PIX_U8, torch.uint16: _lib.PIX_U16, torch.int16: _lib.PIX_U16,
        torch.float32: _lib.PIX_F32}
_STORE_DTYPE = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}

PARAM_KEYS = ("num_levels", "kernel_radius", "iterations", "norm_radius", "norm_eps", "reg_rel", "reg_abs")


def _stream_ptr(device: int) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Handle:
    """Owns an ofv_handle: workspace for up to max_batch pairs of max_width x max_height."""

    def __init__(self, max_width: int, max_height: int, max_batch: int = 1, device: Optional[int] = None):
        lib = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.max_width, self.max_height, self.max_batch = int(max_width), int(max_height), int(max_batch)
        h = c_void_p()
        check(lib.ofv_create(byref(h), self.device, self.max_width, self.max_height, self.max_batch,
                             c_void_p(_stream_ptr(self.device))))
        self._h = h

    @property
    def ptr(self) -> c_void_p:
        if self._h is None:
            raise RuntimeError("handle is closed")
        return self._h

    def bind_stream(self) -> None:
        check(load().ofv_set_stream(self.ptr, c_void_p(_stream_ptr(self.device))), self.ptr)

    def workspace_bytes(self) -> int:
        n = c_size_t()
        check(load().ofv_workspace_bytes(self.ptr, byref(n)), self.ptr)
        return n.value

    def reserve_backward(self, levels: int, iterations: int, pairs: int = 1, store_all: bool = False) -> None:
        """Allocate the adjoint's workspace for batches of up to `pairs` pairs with up to `levels` x
        `iterations`, with the store-all record if asked (set-up call)."""
        mode = _lib.BACKWARD_STORE_ALL if store_all else 0
        check(load().ofv_reserve_backward_ex(self.ptr, int(levels), int(iterations), int(pairs), mode), self.ptr)

    def backward_workspace_bytes(self, levels: int, iterations: int, pairs: int = 1, store_all: bool = False) -> int:
        """Device bytes reserve_backward would allocate for these limits (no allocation)."""
        out = c_size_t()
        mode = _lib.BACKWARD_STORE_ALL if store_all else 0
        check(load().ofv_backward_workspace_bytes(self.ptr, int(levels), int(iterations), int(pairs), mode,
                                                  byref(out)), self.ptr)
        return int(out.value)

    def set_gn_variant(self, variant: str = "auto", tile_h: int = 0) -> None:
        """Force a work decomposition of the Gauss-Newton kernel ('auto', 'march', 'tile64x32', 'tile64x16',
        'tile32x16', 'tile16x16', 'tile64x32w', 'tile64x16w', 'tile64x64', 'tile16x16w', 'tile32x16w', 'tile32x32w')."""
        check(load().ofv_set_gn_variant(self.ptr, _lib.GN_VARIANTS[variant], int(tile_h)), self.ptr)

    def autotune(self, frame0: torch.Tensor, frame1: torch.Tensor, params: Dict, bit_depth: Optional[int] = None,
                 repeats: int = 3) -> torch.Tensor:
        """Time every decomposition on this pair and keep the fastest per level (synchronises)."""
        self.bind_stream()
        h, w = frame0.shape
        out = torch.empty((2, h, w), dtype=torch.float32, device=frame0.device)
        i0, i1 = image_desc(frame0, bit_depth), image_desc(frame1, bit_depth)
        p = params_struct(params)
        check(load().ofv_autotune(self.ptr, byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr()), int(repeats)),
              self.ptr)
        return out

    def autotune_batch(self, frames0: Sequence[torch.Tensor], frames1: Sequence[torch.Tensor], params: Dict,
                       bit_depth: Optional[int] = None, repeats: int = 3) -> List[torch.Tensor]:
        """Time every decomposition on this batch (computed as compute_flow_batch computes it) and keep the
        fastest per launch group (synchronises)."""
        self.bind_stream()
        n = len(frames0)
        outs = [torch.empty((2,) + tuple(f.shape), dtype=torch.float32, device=f.device) for f in frames0]
        arr0 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames0])
        arr1 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames1])
        out_ptrs = (c_void_p * n)(*[o.data_ptr() for o in outs])
        p = params_struct(params)
        check(load().ofv_autotune_batch(self.ptr, n, arr0, arr1, byref(p), out_ptrs, int(repeats)), self.ptr)
        return outs

    def tuning_table(self) -> str:
        need = c_size_t()
        check(load().ofv_tuning_export(self.ptr, None, 0, byref(need)), self.ptr)
        buf = ctypes.create_string_buffer(need.value)
        check(load().ofv_tuning_export(self.ptr, buf, need.value, byref(need)), self.ptr)
        return buf.value.decode()

    def load_tuning_table(self, text: str) -> None:
        check(load().ofv_tuning_import(self.ptr, text.encode()), self.ptr)

    def stream_push(self, frame: torch.Tensor, params: Dict, flow_init: Optional[torch.Tensor] = None,
                    bit_depth: Optional[int] = None, out: Optional[torch.Tensor] = None) -> Optional[torch.Tensor]:
        """Push the next frame of a sequence: the flow from the previous pushed
        frame to this one ([2, H, W]), or None on the first push.  Each frame
        is normalised and reduced once."""
        h, w = frame.shape
        self.bind_stream()
        if out is None:
            out = torch.empty((2, h, w), dtype=torch.float32, device=frame.device)
        _check_flow(out, h, w, "out")
        if flow_init is not None:
            _check_flow(flow_init, h, w, "flow_init")
        img = image_desc(frame, bit_depth)
        p = params_struct(params)
        produced = ctypes.c_int(0)
        check(load().ofv_stream_push(self.ptr, byref(img), byref(p),
                                     c_void_p(flow_init.data_ptr()) if flow_init is not None else None,
                                     c_void_p(out.data_ptr()), byref(produced)), self.ptr)
        return out if produced.value else None

    def stream_reset(self) -> None:
        check(load().ofv_stream_reset(self.ptr), self.ptr)

    def fits(self, w: int, h: int, n: int = 1) -> bool:
        return w <= self.max_width and h <= self.max_height and n <= self.max_batch

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            check(load().ofv_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default: Dict[int, Handle] = {}


def default_handle(w: int, h: int, n: int = 1, device: Optional[int] = None) -> Handle:
    dev = torch.cuda.current_device() if device is None else int(device)
    hd = _default.get(dev)
    if hd is None or not hd.fits(w, h, n):
        mw, mh, mn = w, h, n
        if hd is not None:
            mw, mh, mn = max(w, hd.max_width), max(h, hd.max_height), max(n, hd.max_batch)
            torch.cuda.synchronize(dev)
            hd.close()
        hd = Handle(mw, mh, mn, dev)
        _default[dev] = hd
    hd.bind_stream()
    return hd


def image_desc(t: torch.Tensor, bit_depth: Optional[int] = None) -> OfvImage:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("frames must be 2-D tensors with unit column stride")
    if not t.is_cuda:
        raise ValueError("frames must be device tensors")
    if t.dtype not in _PIX:
        raise ValueError(f"unsupported frame dtype {t.dtype}")
    typ = _PIX[t.dtype]
    if bit_depth is None:
        bit_depth = {torch.uint8: 8, torch.uint16: 16, torch.int16: 16}.get(t.dtype, 0)
    return OfvImage(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0), typ, int(bit_depth))


def params_struct(params: Dict) -> OfvParams:
    p = OfvParams()
    load().ofv_default_params(byref(p))
    for k in PARAM_KEYS:
        if k in params:
            setattr(p, k, params[k])
    st = params.get("storage", "f32")
    p.storage = _lib.STORE[st] if isinstance(st, str) else int(st)
    est = params.get("estimator", "symmetric")
    if est not in ("symmetric", "forward_additive"):
        raise ValueError(f"unknown estimator {est!r}")
    if est == "forward_additive":
        p.flags |= _lib.FLAG_FORWARD_ADDITIVE
    upd = params.get("update", "consistent")
    if upd not in ("consistent", "increment"):
        raise ValueError(f"unknown update {upd!r}")
    if upd == "increment":
        p.flags |= _lib.FLAG_INCREMENT_UPDATE
    if not params.get("fp64_fallback", True):
        p.flags |= _lib.FLAG_NO_FP64_FALLBACK
    if params.get("store_all", False):
        p.flags |= _lib.FLAG_STORE_ALL
    if params.get("save_iterates", False):
        p.flags |= _lib.FLAG_SAVE_ITERATES
    if params.get("saved_forward", False):
        p.flags |= _lib.FLAG_SAVED_FORWARD
    return p


def compute_flow(frame0: torch.Tensor, frame1: torch.Tensor, params: Dict, flow_init: Optional[torch.Tensor] = None,
                 bit_depth: Optional[int] = None, out: Optional[torch.Tensor] = None,
                 handle: Optional[Handle] = None) -> torch.Tensor:
    """Dense flow [2, H, W] float32 (u, v in px/frame) of one pair.  params["save_iterates"] keeps the
    iterates in the handle's backward workspace for a following backward with params["saved_forward"]
    (reserves it first)."""
    h, w = frame0.shape
    hd = handle or default_handle(w, h, 1, frame0.device.index)
    if handle is not None:
        hd.bind_stream()
    if params.get("save_iterates", False):
        hd.reserve_backward(params.get("num_levels", 3), params.get("iterations", 3),
                            store_all=bool(params.get("store_all", False)))
    if out is None:
        out = torch.empty((2, h, w), dtype=torch.float32, device=frame0.device)
    _check_flow(out, h, w, "out")
    i0, i1 = image_desc(frame0, bit_depth), image_desc(frame1, bit_depth)
    p = params_struct(params)
    if flow_init is None:
        st = load().ofv_compute_flow(hd.ptr, byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr()))
    else:
        _check_flow(flow_init, h, w, "flow_init")
        st = load().ofv_compute_flow_ex(hd.ptr, byref(i0), byref(i1), byref(p), c_void_p(flow_init.data_ptr()),
                                        c_void_p(out.data_ptr()))
    check(st, hd.ptr)
    return out


def compute_flow_static(frame0: torch.Tensor, frame1: torch.Tensor, params: Dict, bit_depth: Optional[int] = None,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Dense flow of one pair through ofv_compute_flow_static: no handle and no device allocation by the
    library (its workspace is a static device array of 48 MiB, about 1.5 Mi pixels per pair); enqueued on the
    current torch stream.  Concurrent calls on one device race (they share that array)."""
    h, w = frame0.shape
    if out is None:
        out = torch.empty((2, h, w), dtype=torch.float32, device=frame0.device)
    _check_flow(out, h, w, "out")
    i0, i1 = image_desc(frame0, bit_depth), image_desc(frame1, bit_depth)
    p = params_struct(params)
    with torch.cuda.device(frame0.device):
        st = load().ofv_compute_flow_static(byref(i0), byref(i1), byref(p), c_void_p(out.data_ptr()),
                                            c_void_p(_stream_ptr(frame0.device.index)))
    check(st, None)
    return out


def compute_flow_batch(frames0: Sequence[torch.Tensor], frames1: Sequence[torch.Tensor], params: Dict,
                       flow_init: Optional[Sequence[Optional[torch.Tensor]]] = None, bit_depth: Optional[int] = None,
                       outs: Optional[Sequence[torch.Tensor]] = None, handle: Optional[Handle] = None
                       ) -> List[torch.Tensor]:
    """Dense flows of n pairs (sizes may differ), each stage one launch over all pairs (params["save_iterates"]
    as for compute_flow)."""
    n = len(frames0)
    if n != len(frames1):
        raise ValueError("frames0 and frames1 differ in length")
    mw = max(f.shape[1] for f in frames0)
    mh = max(f.shape[0] for f in frames0)
    hd = handle or default_handle(mw, mh, n, frames0[0].device.index)
    if handle is not None:
        hd.bind_stream()
    if params.get("save_iterates", False):
        hd.reserve_backward(params.get("num_levels", 3), params.get("iterations", 3), pairs=n,
                            store_all=bool(params.get("store_all", False)))
    if outs is None:
        outs = [torch.empty((2,) + tuple(f.shape), dtype=torch.float32, device=f.device) for f in frames0]
    arr0 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames0])
    arr1 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames1])
    out_ptrs = (c_void_p * n)(*[o.data_ptr() for o in outs])
    init_ptrs = None
    if flow_init is not None:
        init_ptrs = (c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in flow_init])
    p = params_struct(params)
    check(load().ofv_compute_flow_batch(hd.ptr, n, arr0, arr1, byref(p), init_ptrs, out_ptrs), hd.ptr)
    return list(outs)


def compute_flow_backward(frame0: torch.Tensor, frame1: torch.Tensor, params: Dict, grad_flow: torch.Tensor,
                          flow_init: Optional[torch.Tensor] = None, bit_depth: Optional[int] = None,
                          need_frames: bool = True, need_init: bool = True, handle: Optional[Handle] = None):
    """Hand-written adjoint: (dL/dframe0, dL/dframe1, dL/dflow_init) for dL/dflow = grad_flow.

    Frame gradients are float32 [H, W] in the frames' own units; entries not
    requested (or dL/dflow_init without flow_init) are None.  params["store_all"] selects the
    store-all mode; params["saved_forward"] skips the forward pass where the handle holds the
    iterates of a saving forward (params["save_iterates"]) on the same inputs.
    """
    h, w = frame0.shape
    hd = handle or default_handle(w, h, 1, frame0.device.index)
    hd.bind_stream()
    hd.reserve_backward(params.get("num_levels", 3), params.get("iterations", 3),
                        store_all=bool(params.get("store_all", False)))
    params = {k: v for k, v in params.items() if k != "save_iterates"}
    _check_flow(grad_flow, h, w, "grad_flow")
    g0 = torch.empty((h, w), dtype=torch.float32, device=frame0.device) if need_frames else None
    g1 = torch.empty((h, w), dtype=torch.float32, device=frame0.device) if need_frames else None
    gi = None
    if flow_init is not None:
        _check_flow(flow_init, h, w, "flow_init")
        if need_init:
            gi = torch.empty((2, h, w), dtype=torch.float32, device=frame0.device)
    i0, i1 = image_desc(frame0, bit_depth), image_desc(frame1, bit_depth)
    p = params_struct(params)
    ptr = lambda t: None if t is None else c_void_p(t.data_ptr())  # noqa: E731
    check(load().ofv_compute_flow_backward(hd.ptr, byref(i0), byref(i1), byref(p), ptr(flow_init), ptr(grad_flow),
                                           ptr(g0), ptr(g1), ptr(gi)), hd.ptr)
    return g0, g1, gi


def compute_flow_backward_batch(frames0: Sequence[torch.Tensor], frames1: Sequence[torch.Tensor], params: Dict,
                                grad_flows: Sequence[torch.Tensor],
                                flow_init: Optional[Sequence[Optional[torch.Tensor]]] = None,
                                bit_depth: Optional[int] = None, need_frames: bool = True, need_init: bool = True,
                                handle: Optional[Handle] = None):
    """The adjoint of n pairs (sizes may differ), each stage one launch over all pairs: lists of
    dL/dframe0, dL/dframe1, dL/dflow_init (None where not requested or without flow_init).
    params["store_all"] selects the store-all mode."""
    n = len(frames0)
    if n != len(frames1) or n != len(grad_flows):
        raise ValueError("frames0, frames1 and grad_flows differ in length")
    mw = max(f.shape[1] for f in frames0)
    mh = max(f.shape[0] for f in frames0)
    hd = handle or default_handle(mw, mh, n, frames0[0].device.index)
    hd.bind_stream()
    hd.reserve_backward(params.get("num_levels", 3), params.get("iterations", 3), pairs=n,
                        store_all=bool(params.get("store_all", False)))
    params = {k: v for k, v in params.items() if k != "save_iterates"}
    dev = frames0[0].device
    g0, g1, gi = [None] * n, [None] * n, [None] * n
    for i in range(n):
        h, w = frames0[i].shape
        _check_flow(grad_flows[i], h, w, "grad_flow")
        if need_frames:
            g0[i] = torch.empty((h, w), dtype=torch.float32, device=dev)
            g1[i] = torch.empty((h, w), dtype=torch.float32, device=dev)
        if flow_init is not None and flow_init[i] is not None:
            _check_flow(flow_init[i], h, w, "flow_init")
            if need_init:
                gi[i] = torch.empty((2, h, w), dtype=torch.float32, device=dev)
    ptrs = lambda ts: (c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in ts])  # noqa: E731
    arr0 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames0])
    arr1 = (OfvImage * n)(*[image_desc(f, bit_depth) for f in frames1])
    p = params_struct(params)
    check(load().ofv_compute_flow_backward_batch(hd.ptr, n, arr0, arr1, byref(p),
                                                 ptrs(flow_init) if flow_init is not None else None,
                                                 ptrs(grad_flows), ptrs(g0) if need_frames else None,
                                                 ptrs(g1) if need_frames else None,
                                                 ptrs(gi) if any(t is not None for t in gi) else None), hd.ptr)
    return g0, g1, gi


class OFVFunction(torch.autograd.Function):
    """Dense flow with gradients w.r.t. both frames and the initial field.

    ``OFVFunction.apply(frame0, frame1, flow_init, params, handle)``; frames
    are float32 [H, W] device tensors (integer frames give no frame
    gradient), flow_init is None or float32 [2, H, W].  The forward keeps its
    iterates in the handle's backward workspace; the backward calls the
    library's hand-written adjoint on them (recompute mode; it re-runs the
    forward itself if another forward on the handle has replaced them).
    """

    @staticmethod
    def forward(ctx, frame0, frame1, flow_init, params, handle=None):
        h, w = frame0.shape
        hd = handle or default_handle(w, h, 1, frame0.device.index)
        # the iterates are kept where the adjoint can use them (its estimator and storage)
        keep = (params.get("storage", "f32") == "f32" and params.get("estimator", "symmetric") == "symmetric"
                and params.get("update", "consistent") == "consistent")
        out = compute_flow(frame0, frame1, dict(params, save_iterates=keep), flow_init=flow_init, handle=hd)
        ctx.params = dict(params, saved_forward=keep)
        ctx.handle = hd
        ctx.has_init = flow_init is not None
        ctx.save_for_backward(frame0, frame1, flow_init if flow_init is not None else frame0.new_empty(0))
        return out

    @staticmethod
    def backward(ctx, grad):
        f0, f1, fi = ctx.saved_tensors
        need_f = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        need_i = ctx.has_init and ctx.needs_input_grad[2]
        g0, g1, gi = compute_flow_backward(f0, f1, ctx.params, grad.contiguous(),
                                           flow_init=fi if ctx.has_init else None, need_frames=need_f,
                                           need_init=need_i, handle=ctx.handle)
        return (g0 if ctx.needs_input_grad[0] else None, g1 if ctx.needs_input_grad[1] else None,
                gi if need_i else None, None, None)


def _check_flow(t: torch.Tensor, h: int, w: int, name: str) -> None:
    if t.dtype != torch.float32 or tuple(t.shape) != (2, h, w) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape (2, {h}, {w})")


# ---------------------------------------------------------------- stage entry points (include/ofv_stages.h)

def _plane_check(t: torch.Tensor, dtype=None):
    if t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError("planes must be 2-D device tensors with unit column stride")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")


def _stage_handle(t: torch.Tensor, handle: Optional[Handle]) -> Handle:
    hd = handle or default_handle(1, 1, 1, t.device.index)
    hd.bind_stream()
    return hd


def stage_normalize(frame: torch.Tensor, norm_radius: int, norm_eps: float, storage: str = "f32",
                    bit_depth: Optional[int] = None, handle: Optional[Handle] = None) -> torch.Tensor:
    hd = _stage_handle(frame, handle)
    h, w = frame.shape
    out = torch.empty((h, w), dtype=_STORE_DTYPE[storage], device=frame.device)
    img = image_desc(frame, bit_depth)
    check(load().ofv_stage_normalize(hd.ptr, byref(img), norm_radius, norm_eps, _lib.STORE[storage],
                                     c_void_p(out.data_ptr()), out.stride(0)), hd.ptr)
    return out


def stage_reduce(plane: torch.Tensor, handle: Optional[Handle] = None) -> torch.Tensor:
    _plane_check(plane)
    storage = {v: k for k, v in _STORE_DTYPE.items()}[plane.dtype]
    hd = _stage_handle(plane, handle)
    h, w = plane.shape
    out = torch.empty(((h + 1) // 2, (w + 1) // 2), dtype=plane.dtype, device=plane.device)
    check(load().ofv_stage_reduce(hd.ptr, _lib.STORE[storage], c_void_p(plane.data_ptr()), w, h, plane.stride(0),
                                  c_void_p(out.data_ptr()), out.stride(0)), hd.ptr)
    return out


def stage_pyramid(plane: torch.Tensor, levels: int, handle: Optional[Handle] = None) -> List[torch.Tensor]:
    """`levels` (1..3) successive REDUCE levels of `plane` in one launch;
    equals chained `stage_reduce` calls bit for bit."""
    _plane_check(plane)
    storage = {v: k for k, v in _STORE_DTYPE.items()}[plane.dtype]
    hd = _stage_handle(plane, handle)
    h, w = plane.shape
    outs = []
    for _ in range(max(int(levels), 1)):
        h, w = (h + 1) // 2, (w + 1) // 2
        outs.append(torch.empty((h, w), dtype=plane.dtype, device=plane.device))
    n = len(outs)
    ptrs = (c_void_p * n)(*[o.data_ptr() for o in outs])
    pitches = (c_int64 * n)(*[o.stride(0) for o in outs])
    check(load().ofv_stage_pyramid(hd.ptr, _lib.STORE[storage], c_void_p(plane.data_ptr()), plane.shape[1],
                                   plane.shape[0], plane.stride(0), int(levels), ptrs, pitches), hd.ptr)
    return outs


def stage_restrict_flow(flow: torch.Tensor, handle: Optional[Handle] = None) -> torch.Tensor:
    _, h, w = flow.shape
    _check_flow(flow, h, w, "flow")
    hd = _stage_handle(flow, handle)
    out = torch.empty((2, (h + 1) // 2, (w + 1) // 2), dtype=torch.float32, device=flow.device)
    check(load().ofv_stage_restrict_flow(hd.ptr, c_void_p(flow.data_ptr()), w, h, w, c_void_p(out.data_ptr()),
                                         (w + 1) // 2), hd.ptr)
    return out


def stage_upsample(flow: torch.Tensor, h: int, w: int, handle: Optional[Handle] = None) -> torch.Tensor:
    _, ch, cw = flow.shape
    _check_flow(flow, ch, cw, "flow")
    hd = _stage_handle(flow, handle)
    out = torch.empty((2, h, w), dtype=torch.float32, device=flow.device)
    check(load().ofv_stage_upsample(hd.ptr, c_void_p(flow.data_ptr()), cw, ch, cw, c_void_p(out.data_ptr()), w, h,
                                    w), hd.ptr)
    return out


def stage_gn_iteration(p0: torch.Tensor, p1: torch.Tensor, flow_in: Optional[torch.Tensor], mode: str,
                       kernel_radius: int, reg_rel: float = 1e-3, reg_abs: float = 1e-9,
                       handle: Optional[Handle] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One fused Gauss-Newton iteration; mode is 'zero', 'direct' or 'upsample'.  out: an optional
    [2, H, W] float32 result buffer (contiguous, not overlapping flow_in)."""
    _plane_check(p0)
    _plane_check(p1, p0.dtype)
    if p1.stride(0) != p0.stride(0) or p1.shape != p0.shape:
        raise ValueError("p0 and p1 must share shape and pitch")
    storage = {v: k for k, v in _STORE_DTYPE.items()}[p0.dtype]
    h, w = p0.shape
    m = {"zero": _lib.FLOW_IN_ZERO, "direct": _lib.FLOW_IN_DIRECT, "upsample": _lib.FLOW_IN_UPSAMPLE}[mode]
    hd = _stage_handle(p0, handle)
    if out is None:
        out = torch.empty((2, h, w), dtype=torch.float32, device=p0.device)
    elif out.dtype != torch.float32 or tuple(out.shape) != (2, h, w) or not out.is_contiguous() or \
            out.device != p0.device:
        raise ValueError("out must be a contiguous [2, H, W] float32 tensor on the planes' device")
    elif flow_in is not None:
        a0, a1 = out.data_ptr(), out.data_ptr() + out.numel() * 4
        b0 = flow_in.data_ptr()
        b1 = b0 + (flow_in.stride(0) * (flow_in.shape[0] - 1) + flow_in.stride(1) * (flow_in.shape[1] - 1) +
                   flow_in.shape[2]) * flow_in.element_size()
        if a0 < b1 and b0 < a1:
            raise ValueError("out overlaps flow_in")
    if flow_in is None:
        fin, iw, ih = None, w, h
    else:
        _, ih, iw = flow_in.shape
        _check_flow(flow_in, ih, iw, "flow_in")
        fin = c_void_p(flow_in.data_ptr())
    check(load().ofv_stage_gn_iteration(hd.ptr, _lib.STORE[storage], c_void_p(p0.data_ptr()),
                                        c_void_p(p1.data_ptr()), w, h, p0.stride(0), m, fin, iw, ih, iw,
                                        c_void_p(out.data_ptr()), w, kernel_radius, reg_rel, reg_abs), hd.ptr)
    return out


def derived(flow: torch.Tensor, mask: Optional[torch.Tensor] = None, dx: float = 1.0, dz: float = 1.0,
            dt: float = 1.0, streamwise_sign: int = 1, probes: Optional[torch.Tensor] = None,
            vorticity: bool = True, area: bool = True, handle: Optional[Handle] = None) -> Dict:
    """Live derived quantities of a [2, H, W] float32 flow in one kernel launch:
    {'vorticity': [H, W] float32 or None, 'area': [1] float64 (recirculation
    area of Eq. RA) or None, 'probes': [n, 2] float32 or None}.  mask: [H, W]
    uint8, 0 = masked.  probes: [n, 2] float32 points (x, y) in pixels."""
    if flow.dim() != 3 or flow.shape[0] != 2 or flow.dtype != torch.float32 or not flow.is_cuda:
        raise ValueError("flow must be a [2, H, W] float32 CUDA tensor")
    if flow.stride(2) != 1 or flow.stride(0) != flow.shape[1] * flow.stride(1):
        raise ValueError("flow planes must be row-major with the v plane height * pitch after the u plane")
    _, h, w = flow.shape
    hd = _stage_handle(flow, handle)
    prm = OfvDerivedParams()
    load().ofv_default_derived_params(byref(prm))
    prm.dx, prm.dz, prm.dt, prm.streamwise_sign = float(dx), float(dz), float(dt), int(streamwise_sign)
    mptr, mpitch = None, 0
    if mask is not None:
        if mask.dtype != torch.uint8 or mask.shape != (h, w) or mask.stride(1) != 1 or mask.device != flow.device:
            raise ValueError("mask must be an [H, W] uint8 tensor with unit column stride on the flow's device")
        mptr, mpitch = c_void_p(mask.data_ptr()), mask.stride(0)
    om = torch.empty((h, w), dtype=torch.float32, device=flow.device) if vorticity else None
    ar = torch.empty(1, dtype=torch.float64, device=flow.device) if area else None
    n = 0
    pxy = puv = None
    if probes is not None:
        pxy = probes.to(device=flow.device, dtype=torch.float32).contiguous().reshape(-1, 2)
        n = pxy.shape[0]
        puv = torch.empty((n, 2), dtype=torch.float32, device=flow.device)
    check(load().ofv_derived(hd.ptr, c_void_p(flow.data_ptr()), w, h, flow.stride(1), mptr, mpitch, byref(prm),
                             c_void_p(om.data_ptr()) if om is not None else None, w,
                             c_void_p(pxy.data_ptr()) if n else None, n,
                             c_void_p(puv.data_ptr()) if n else None,
                             c_void_p(ar.data_ptr()) if ar is not None else None), hd.ptr)
    return {"vorticity": om, "area": ar, "probes": puv if n else None}
