"""Seeded synthetic inputs for velocity-gauge real-time TDDFTB propagation.

This module builds the *inputs* of the propagation and nothing else:
crystal / amorphous geometries, the real-space two-centre Slater-Koster
blocks H0(I,J,L) and S(I,J,L) with their bond vectors, Gamma-centred k-point
meshes, the Ewald-free gamma matrix, and the vector-potential drive tables.
It performs no Bloch sum, no Mulliken analysis, no ground-state solve and no
time stepping: those belong to the method, which the HIP library and the
CPU oracle each implement on their own.

Units are atomic units (bohr, hartree, atomic time); c = 137.035999084.
"""
from .systems import (  # noqa: F401
    TBSystem,
    C_LIGHT,
    FS_AU,
    diamond_supercell,
    amorphous_si,
    linear_chain,
    random_cell,
    random_hermitian_density,
    primitive_diamond,
    gamma_mesh,
    config_system,
    CONFIGS,
)
from .fields import kick_table, sin2_pulse_table  # noqa: F401
