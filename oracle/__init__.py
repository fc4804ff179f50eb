"""FP64 CPU oracle (test infrastructure only; never used by the product path).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It shares no code with the HIP library.
"""
from .ofv_oracle import (compute_flow, normalize, intensity, reduce, pyramid, bilinear,
                         central_gradient, warp_terms, gn_iteration, upsample, restrict_flow,
                         window_sum, endpoint_error, Trace, DEFAULTS, BINOMIAL5)
from .ofv_derived import vorticity, recirculation_area, probes, ddi, ddj

__all__ = ["compute_flow", "normalize", "intensity", "reduce", "pyramid", "bilinear",
           "central_gradient", "warp_terms", "gn_iteration", "upsample", "restrict_flow",
           "window_sum", "endpoint_error", "Trace", "DEFAULTS", "BINOMIAL5",
           "vorticity", "recirculation_area", "probes", "ddi", "ddj"]
