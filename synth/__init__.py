"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This package holds no arithmetic of the Monte Carlo method itself: it only
builds lattices (CSR neighbour lists with per-bond exchange constants, per-site
anisotropy constants and axes, per-site field directions), temperature/field
schedules and spin configurations, all drawn from SplitMix64 (Steele, Lea and
Flood, OOPSLA 2014) so that the inputs do not depend on numpy's own generators.

The lattice description follows the material file of the paper (section
"Material building"): sites, exchange links with their constants, a field axis
per site, and the anisotropy file's per-site constant and axis.
"""
from .splitmix import splitmix64, uniform01, normal01, unit_vectors
from .lattices import (Lattice, sc_periodic, from_bonds, isolated, open_chain,
                       random_tree, core_shell_ball, diluted_film, film_batch,
                       gradient_lattice, random_spins)
from .schedules import cooling_schedule, replica_temperatures, hysteresis_fields

__all__ = [
    "splitmix64", "uniform01", "normal01", "unit_vectors", "Lattice",
    "sc_periodic", "from_bonds", "isolated", "open_chain", "random_tree",
    "core_shell_ball", "diluted_film", "film_batch", "gradient_lattice",
    "random_spins", "cooling_schedule", "replica_temperatures",
    "hysteresis_fields",
]
