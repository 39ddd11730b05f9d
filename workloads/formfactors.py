"""Invented electron form-factor coefficients.

The paper delegates the atomic potentials to its multislice programs and prints no
parametrisation.  The functional form used here is the common sum of three Lorentzian and three
Gaussian terms,

    f(q) = sum_i a_i / (q^2 + b_i) + sum_i c_i exp(-d_i q^2)      (q in 1/Angstrom, f in Angstrom)

with coefficients that are *made up* for this project (they are not any real element's
tabulated values).  They give a realistic weak-to-moderate phase per atom at 60-100 keV.

Row layout, shared by every consumer: a1, b1, a2, b2, a3, b3, c1, d1, c2, d2, c3, d3.
"""
import numpy as np

_A = np.array([0.30, 0.15, 0.20, 1.5, 0.05, 10.0,
               0.40, 3.0, 0.15, 0.6, 0.02, 0.1], dtype=np.float64)


def _scaled(base, amp, dscale=1.0):
    out = base.copy()
    out[[0, 2, 4, 6, 8, 10]] *= amp          # a_i and c_i carry the amplitude
    out[[7, 9, 11]] *= dscale                # d_i (Gaussian widths)
    return out


FORM_FACTORS = {
    "A": _A,
    "B": _scaled(_A, 0.6),
    "BN-B": _scaled(_A, 0.8),
    "BN-N": _scaled(_A, 0.9, dscale=0.9),
    # single-Gaussian test species used by the closed-form potential check
    "gauss-test": np.array([0, 1, 0, 1, 0, 1, 1.0, 6.25, 0, 1, 0, 1], dtype=np.float64),
    # single-Lorentzian test species used by the K0 closed-form check
    "lorentz-test": np.array([0.5, 0.15, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1], dtype=np.float64),
}


def form_factor_table(names):
    """Stack coefficient rows for the given species names -> float64 [n_species][12]."""
    return np.stack([FORM_FACTORS[n] for n in names]).astype(np.float64)
