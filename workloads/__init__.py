"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only *synthesises inputs*: atom positions along a time-ordered trajectory,
species ids, invented form-factor coefficients and the parameters of each workload.  It holds
none of the method's arithmetic (no potentials, no propagation, no spectra), so both the CPU
oracle and the GPU path can consume exactly the same arrays without sharing any code.

The paper's inputs are molecular-dynamics trajectories (the two-step procedure: an MD run, then
multislice through every snapshot).  No MD engine or trained interatomic potential is available
here, so a superposition of harmonic phonon modes stands in for the trajectory: it has the same
shape ([T][N_atoms][3], float32 Angstrom), strongly correlated consecutive snapshots and
vibrational energies below the Nyquist energy pi*hbar/dt of the sampling.
"""
from .formfactors import FORM_FACTORS, form_factor_table
from .structures import Structure, fcc_cubic, rocksalt, hexagonal_bn_like
from .trajectory import harmonic_trajectory, static_trajectory, rigid_shift_trajectory
from .configs import CONFIGS, Workload, make_workload

__all__ = [
    "FORM_FACTORS", "form_factor_table", "Structure", "fcc_cubic", "rocksalt", "hexagonal_bn_like",
    "harmonic_trajectory", "static_trajectory", "rigid_shift_trajectory", "CONFIGS", "Workload",
    "make_workload",
]
