"""FP64 CPU oracle for the time auto-correlation (TACAW) hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the benchmark's CPU
baseline leg may import this package.  The product path (the C-ABI library and its binding)
never calls it and shares no code with it.

Everything here is written for a reader holding the paper: plain definitions, complex128 and
float64, dense DFT matrices instead of FFTs, and no blocking or fusion.  Each function cites the
passage of the paper it follows.  The paper delegates the multislice internals to external
programs, so those follow the textbook multislice method; the readings taken where the paper is
silent are listed in the design notes and repeated in the docstrings.

Modules:
  physics    - constants, relativistic wavelength and interaction parameter, energy axis, Kubo factor
  dft        - dense DFT matrices
  potential  - slice binning, form factors, band limit, projected slice potentials
  multislice - initial waves, transmission/propagation, exit-wave stack
  spectrum   - segment periodograms, brute-force correlation, Kubo correction, normalisation
  adjoint    - hand-written FP64 adjoints (spectrum, multislice, atom positions)
"""
from . import physics, dft, potential, multislice, spectrum, adjoint  # noqa: F401
