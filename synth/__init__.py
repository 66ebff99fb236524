"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input generation: closed triangle meshes of the
obstacles (the boundary meshes the cut-cell construction consumes), velocity
fields sampled at vertex positions, seeded particle sets, and the named
workload definitions.  It
contains none of the method's arithmetic (no cut cells, no VEM, no multigrid).
"""
from .shapes import icosphere, ellipsoid, box, plate_pair, thin_sheet, mesh_area
from .fields import normal_field, fourier_field
from .configs import CONFIGS, get_config, Workload
from .particles import seeded_particles

__all__ = [
    "icosphere", "ellipsoid", "box", "plate_pair", "thin_sheet", "mesh_area",
    "normal_field", "fourier_field", "CONFIGS", "get_config", "Workload", "seeded_particles",
]
