"""Seeded synthetic inputs: particle-image pairs and their analytic flows.

Input generation only: nothing here computes any part of the flow estimator.
"""
from .particles import ParticlePair, make_pair, make_stripes_pair, make_texture, render_particles, FWHM_PER_SIGMA
from .flows import Translation, Rankine, Turbulence, CylinderWake
from .configs import (config_rankine_256, config_shear_1mp, config_turbulence_4mp,
                      config_adjoint_512, config_paper_sweep, WORKLOADS)

__all__ = [
    "ParticlePair", "make_pair", "make_stripes_pair", "make_texture", "render_particles", "FWHM_PER_SIGMA",
    "Translation", "Rankine", "Turbulence", "CylinderWake",
    "config_rankine_256", "config_shear_1mp", "config_turbulence_4mp", "config_adjoint_512",
    "config_paper_sweep", "WORKLOADS",
]
