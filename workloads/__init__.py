"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds input recipes only: velocity models, acquisition geometry,
search boxes and particle draws. It contains none of the method's arithmetic
(no stencil, no interpolation, no time stepping, no misfit, no stability limit),
and it imports nothing from the oracle or from the HIP package.
"""
from .models import two_layer, layered_faulted, uniform_particles
from .configs import config, CONFIG_NAMES

__all__ = ["two_layer", "layered_faulted", "uniform_particles", "config", "CONFIG_NAMES"]
