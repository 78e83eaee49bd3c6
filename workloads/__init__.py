"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

Holds inputs only (operators, states, time grids); no part of the method.
"""
from .systems import (Op, System, dense, diag, csr_from_dense, csr_from_triplets,  # noqa: F401
                      two_level, unitary_example, two_channel_identity, jaynes_cummings,
                      tfim, random_system, hetero_batch, photon_birth_death, trilinear,
                      by_name, destroy, coherent_amplitudes, driven_two_level, commuting_drive,
                      driven_jaynes_cummings)
