"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random numbers and lays out atoms: lattices, displacement
fields, defects, Maxwell velocities, random coefficient vectors and the integer
enumeration of the ACE basis index list. It contains none of the arithmetic of
the adaptive-precision method (no potentials, no descriptors, no switching).
"""
from .structures import (bcc, fcc, gaussian_displace, screw_dipole_z, local_noise,
                         remove_atoms, vacancy_clusters, penny_crack, maxwell_velocities,
                         strain_cell, dilatation_inclusion, frenkel_pairs)
from .basis import ace_basis, basis_counts
from .configs import load_config, build_system, CONFIG_NAMES
from . import learned

__all__ = ["bcc", "fcc", "gaussian_displace", "screw_dipole_z", "local_noise", "remove_atoms",
           "vacancy_clusters", "penny_crack", "maxwell_velocities", "strain_cell", "ace_basis",
           "basis_counts", "dilatation_inclusion", "frenkel_pairs", "load_config", "build_system", "CONFIG_NAMES"]
