"""The seeded synthetic workloads, with their estimator parameters as plain data.

Each builder returns ``(pair, params)``: a :class:`ParticlePair` and a dict
with every estimator parameter spelled out (pyramid levels = PSL + 1, window
radius KR, Gauss-Newton iterations IT per level, normalisation radius NR,
normalisation epsilon, damping constants and image storage).  Callers pass
these values explicitly to whichever implementation they exercise.

Workloads (frame size, pixel type, particles, flow, parameters):

* ``rankine_256``  256x256 8-bit, FWHM 2.5 px, 0.1 ppp, A ~ U(0.5, 1) * 255,
  noise sigma 2 DN, Rankine vortex R = 32 px, D = 3 px centred at
  ((W-1)/2, (H-1)/2); 3 levels, KR 4, IT 3, NR 1.
* ``shear_1mp``    1024x1024 12-bit in uint16, FWHM 2.2 px, 0.08 ppp,
  noise 1 % of full scale, translation (1.37, -0.62) px plus du/dy = 0.01
  about the centre row; 4 levels, KR 5, IT 4, NR 1.
* ``turbulence_4mp`` 2048x2048 12-bit, FWHM 2.5 px, 0.1 ppp, 1 % noise,
  256-mode k^-5/3 divergence-free field, RMS 2 px, max <= 8 px, pair t of a
  time-resolved sequence (seed 3000 + t); 5 levels, KR 4, IT 3, NR 2.
* ``adjoint_512``  512x512 float32 frames, noise 2/255, Rankine (R 32,
  D 3, seeded centre) for even i and a turbulence crop for odd i; 3 levels,
  KR 4, IT 3, NR 1.
* ``paper_sweep``  8-bit pairs at the paper's throughput setting
  (NR 2, KR 10, IT 3, PSL 0..2 i.e. 1..3 levels; section "Post-processing
  (offline) performances").
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .flows import Rankine, Translation, Turbulence
from .particles import ParticlePair, make_pair

# Parameter values shared by every workload (the readings of the method's
# unstated constants; both implementations receive them as explicit inputs).
_COMMON = {"norm_eps": 1e-4, "reg_rel": 1e-3, "reg_abs": 1e-9, "storage": "f32"}


def _params(levels: int, kr: int, it: int, nr: int, **kw) -> Dict:
    p = {"num_levels": levels, "kernel_radius": kr, "iterations": it, "norm_radius": nr}
    p.update(_COMMON)
    p.update(kw)
    return p


def config_rankine_256(seed: int = 1, size: int = 256) -> Tuple[ParticlePair, Dict]:
    c = (size - 1) / 2.0
    pair = make_pair(size, size, Rankine(c, c, 32.0, 3.0), fwhm=2.5, ppp=0.1, seed=seed,
                     bit_depth=8, noise=2.0)
    return pair, _params(3, 4, 3, 1)


def config_shear_1mp(seed: int = 2, size: int = 1024) -> Tuple[ParticlePair, Dict]:
    flow = Translation(1.37, -0.62, shear=0.01, y_ref=(size - 1) / 2.0)
    pair = make_pair(size, size, flow, fwhm=2.2, ppp=0.08, seed=seed, bit_depth=12,
                     noise=0.01 * 4095.0)
    return pair, _params(4, 5, 4, 1)


def config_turbulence_4mp(t: int = 0, size: int = 2048, field_seed: int = 3) -> Tuple[ParticlePair, Dict]:
    flow = Turbulence(seed=field_seed, rms=2.0, dmax_cap=8.0, ref_h=256, ref_w=256, t=float(t))
    pair = make_pair(size, size, flow, fwhm=2.5, ppp=0.1, seed=3000 + t, bit_depth=12,
                     noise=0.01 * 4095.0)
    return pair, _params(5, 4, 3, 2, storage="f16")


def config_adjoint_512(i: int = 0, size: int = 512) -> Tuple[ParticlePair, Dict]:
    rng = np.random.default_rng(6000 + i)
    if i % 2 == 0:
        cx, cy = rng.uniform(0.3 * size, 0.7 * size, 2)
        flow = Rankine(cx, cy, 32.0, 3.0)
    else:
        flow = Turbulence(seed=6000 + i, rms=2.0, dmax_cap=8.0, ref_h=128, ref_w=128)
    pair = make_pair(size, size, flow, fwhm=2.5, ppp=0.1, seed=6000 + i, bit_depth=0,
                     noise=2.0 / 255.0)
    return pair, _params(3, 4, 3, 1)


def config_paper_sweep(h: int = 1024, w: int = 1024, levels: int = 3, i: int = 0) -> Tuple[ParticlePair, Dict]:
    flow = Turbulence(seed=5000 + i, rms=2.0, dmax_cap=8.0, ref_h=256, ref_w=256)
    pair = make_pair(h, w, flow, fwhm=2.5, ppp=0.1, seed=5000 + i, bit_depth=8, noise=2.0)
    return pair, _params(levels, 10, 3, 2)


WORKLOADS = {
    "rankine_256": config_rankine_256,
    "shear_1mp": config_shear_1mp,
    "turbulence_4mp": config_turbulence_4mp,
    "adjoint_512": config_adjoint_512,
    "paper_sweep": config_paper_sweep,
}
