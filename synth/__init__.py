"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no gravity arithmetic: it only draws density models,
station samples and request traces from seeded generators, so that the CPU
oracle and the HIP path see bit-identical inputs.  Densities are returned in
kg/m^3 (the paper's unit for the validation model, section 3.1), laid out
``[nz][ny][nx]`` with x fastest, the index order of the paper's cell
numbering (section 2.2).
"""

from .geometry import Geometry, PRESETS, paper_e1_geometry
from .density import (
    tiny_density,
    prisms_and_grf,
    random_prisms,
    gaussian_random_field,
    batch_density,
    paper_e1_density,
    sample_stations,
    sample_cells,
)
from .trace import poisson_trace

__all__ = [
    "Geometry",
    "PRESETS",
    "paper_e1_geometry",
    "tiny_density",
    "prisms_and_grf",
    "random_prisms",
    "gaussian_random_field",
    "batch_density",
    "paper_e1_density",
    "sample_stations",
    "sample_cells",
    "poisson_trace",
]
