"""Seeded synthetic inputs shaped like single-particle-imaging (SPI) workloads.

This module draws random numbers and lays out inputs; it holds none of the
slicing, matching or spreading arithmetic.  Both the CPU oracle and the GPU
library consume what it returns, and neither is imported here.

Everything is deterministic in ``(config, role)``: each role owns one
``numpy.random.Generator`` seeded from ``SeedSequence([config, role])`` and
draws sequentially, so the first ``k`` rows of any per-image or
per-orientation array do not depend on how many rows were requested.
"""
from .generators import (  # noqa: F401
    CONFIGS, ROLE, Config, config, rng, molecule, intensity_model, detector_q,
    quaternions, poisson_counts, pixel_weights, complex_perturbation,
    fd_voxels, photon_scale, random_points, random_model,
)
