"""Seeded synthetic inputs for the dense OMM path (test and benchmark infrastructure).

This package builds the matrices the method is *given*: the overlap S, the kinetic matrix T, the
Hamiltonian H of a finite-range model basis, and a random starting coefficient matrix C0. It holds
none of the minimization's arithmetic, and both the CPU oracle and the HIP path receive exactly the
arrays it returns.
"""

from .generator import (  # noqa: F401
    CONFIGS,
    System,
    batched_systems,
    bloch_system,
    complex_start_coefficients,
    config_system,
    lattice_positions,
    make_system,
    perturb_hamiltonian,
    start_coefficients,
)
