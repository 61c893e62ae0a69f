"""Seeded synthetic workloads shared by the HIP path, the oracle and the benchmark.

This package holds problem set-ups only (grid sizes, boundary kinds, dimensionless
groups converted to lattice units, initial and forcing fields, inlet profiles and the
seeded draws of the batched and adjoint workloads).  It contains none of the lattice
Boltzmann arithmetic: relaxation times, equilibria, collisions and boundary schemes are
implemented separately by the library and by the oracle.
"""
from .workloads import (  # noqa: F401
    Problem,
    Problem3D,
    random3d,
    channel3d,
    lattice_units,
    poiseuille,
    four_roll_mill,
    cylinder,
    cylinder_channel,
    batch_c4,
    adjoint_c5,
    smooth_force_perturbation,
    rest_state,
    random_periodic,
    waves,
)
