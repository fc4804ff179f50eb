"""The benchmark's algorithmic byte models (host arithmetic only, no GPU).

The per-sweep model prices every Gauss-Newton iteration at its level's two
image planes and the flow in and out; the hot-path measurement plan tabulates
its bytes per vector for each workload, which pins the model here.  The
fused-iteration bound is the same model with one iteration per level."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("name,levels,w,h,iters,s_bytes,in_bytes,per_vec", [
    ("256^2 u8 Rankine, FP32", 3, 256, 256, 3, 4, 1, 109.0),
    ("1024^2 12-bit shear, FP32", 4, 1024, 1024, 4, 4, 2, 144.625),
    ("2048^2 12-bit turbulence, FP16", 5, 2048, 2048, 3, 2, 2, 86.5625),
    ("5120x4096 8-bit, three levels, FP32", 3, 5120, 4096, 3, 4, 1, 109.0),
])
def test_per_sweep_bytes_per_vector(name, levels, w, h, iters, s_bytes, in_bytes, per_vec):
    assert bench._sweep_bytes(levels, w, h, iters, s_bytes, in_bytes) == pytest.approx(per_vec * w * h, rel=1e-12)


def test_live_step_bytes():
    """The live step (5120x4096 with 2048^2 and 1024^2 crops, BF16 planes, L 4, IT 3): 2.26 GB."""
    total = sum(bench._sweep_bytes(4, w, h, 3, 2, 2) for w, h in ((5120, 4096), (2048, 2048), (1024, 1024)))
    assert total == pytest.approx(2.26e9, rel=2e-3)


def test_fused_iteration_bound():
    """One iteration per level: each further iteration adds 2 s + 16 bytes per level pixel."""
    per, fused = bench._sweep_bytes(4, 1024, 1024, 4, 4, 2), bench._sweep_bytes(4, 1024, 1024, 1, 4, 2)
    px = sum(((1024 + (1 << l) - 1) >> l) ** 2 for l in range(4))
    assert per - fused == 3 * (2 * 4 + 16) * px
    m = bench._step_models(per, fused, 1e-4)
    assert m["per_sweep"]["frac_of_8TBps"] == round(per / 1e-4 / 8e12, 4)
    assert m["fused_iterations"]["bytes"] == fused < per
