"""Dense optical-flow velocimetry on AMD Instinct MI355X (gfx950).

The estimator of arXiv 2509.25924 (symmetric, pyramidal, iterative
Lucas-Kanade) runs entirely in the HIP kernels of ``libofv.so`` behind the
C ABI in ``include/ofv.h``; this package only marshals torch tensors into
those calls.
"""
from .api import (Handle, OFVFunction, compute_flow, compute_flow_backward, compute_flow_backward_batch, compute_flow_batch, compute_flow_static, default_handle,
                  stage_gn_iteration, stage_normalize, stage_pyramid, derived, stage_reduce, stage_restrict_flow, stage_upsample)
from ._lib import OfvError, load

__all__ = ["Handle", "OFVFunction", "compute_flow", "compute_flow_backward", "compute_flow_backward_batch", "compute_flow_batch", "compute_flow_static", "default_handle", "stage_gn_iteration",
           "stage_normalize", "stage_pyramid", "derived", "stage_reduce", "stage_restrict_flow", "stage_upsample", "OfvError", "load"]
