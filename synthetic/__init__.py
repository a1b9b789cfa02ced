"""Seeded synthetic spin-orbital Hamiltonians.

This package only draws random numbers and arranges them into the input
format (a Fock matrix and antisymmetrized two-electron integrals).  It holds
none of the coupled-cluster arithmetic; both the CPU oracle and the GPU
library consume its output bytes.
"""
from .hamiltonian import (SyntheticHamiltonian, make_hamiltonian, config_hamiltonian,
                          CONFIGS, batch_instance_shapes, full_virtuals_for)

__all__ = ["SyntheticHamiltonian", "make_hamiltonian", "config_hamiltonian", "CONFIGS",
           "batch_instance_shapes", "full_virtuals_for"]
