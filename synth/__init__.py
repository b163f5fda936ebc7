"""Seeded synthetic spinor inputs shared by the oracle and the GPU path.

This package builds inputs only: G-spheres, random orthonormal two-component
spinor coefficients, band energies, imaginary frequencies and the bare Coulomb
potential the caller hands to the epsilon stage, and a valence charge density
for the plasmon-pole model.  It holds none of the
polarizability arithmetic (no transforms, no products, no contraction, no
inversion), so the oracle and the HIP path stay independent of each other.
"""
from .generate import (  # noqa: F401
    CONFIGS,
    SystemConfig,
    build_system,
    g_sphere,
    config_by_name,
    config_digest,
    batch_systems,
    closure_systems,
    EV_PER_HA,
    charge_density,
    vcoul,
)
