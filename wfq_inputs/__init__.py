"""Seeded synthetic inputs shared by the oracle tests, the device tests and the benchmark.

This package holds only input recipes: lattice geometries, seeded positional
jitter and the workload descriptions (sizes, frequency grids, parameter
values). It contains none of the method's arithmetic (no interaction kernel,
no Laplacian, no solver), so that the oracle and the device path share
nothing but their inputs.
"""

from .rng import splitmix64, uniform01, gaussian
from .geometry import (
    graphene_disk,
    graphene_sheet,
    graphene_ribbon,
    nanotube,
    nanotube_atoms_per_cell,
    nanotube_diameter,
    fcc_sphere,
    jitter,
    A_CC,
    A_GRAPHENE,
    A_FCC,
)
from .workloads import Workload, workload, WORKLOADS, sub_window, serve_mix_jobs

__all__ = [
    "splitmix64", "uniform01", "gaussian",
    "graphene_disk", "graphene_sheet", "graphene_ribbon", "nanotube",
    "nanotube_atoms_per_cell", "nanotube_diameter", "fcc_sphere", "jitter",
    "A_CC", "A_GRAPHENE", "A_FCC",
    "Workload", "workload", "WORKLOADS", "sub_window", "serve_mix_jobs",
]
