"""Seeded synthetic initial states for the short-range MD workloads.

This module holds only input generation (lattices, random placement, random
velocities).  It contains none of the pair-force, neighbour-list or integrator
arithmetic, so both the CPU oracle tests and the GPU path can draw their inputs
from it without sharing any of the method's code.
"""
from .generators import (  # noqa: F401
    State,
    KA_SIGMA,
    KA_EPSILON,
    fcc_lattice,
    lj_fcc_state,
    ka_random_state,
    ka_replica_states,
    maxwell_boltzmann,
    jitter_positions,
    lj_params,
    ka_params,
    config0_state,
    config1_state,
    config2_state,
    config3_states,
    config4_state,
)
