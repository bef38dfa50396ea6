"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds workload descriptions (cylinder radius, axial period, twist,
cutoff, grid sizes), seeded atom layouts for Gaussian-well model potentials,
sampling of such a potential at given helical-coordinate points, and seeded
random coefficient blocks.  It contains none of the helical-wave method's
arithmetic (no basis functions, quadrature, transforms or Hamiltonian): both
the CPU oracle and the GPU library receive what is generated here as input.
"""
from .configs import Workload, WORKLOADS, workload  # noqa: F401
from .structures import atoms_for, potential_at, cyclic_images, Atom  # noqa: F401
from .blocks import random_block  # noqa: F401
