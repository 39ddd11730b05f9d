"""Physical constants and scalar relations (oracle, FP64).

Constants (CODATA 2018):
  hc        = 12398.419843320026 eV*Angstrom
  m0 c^2    = 510998.95 eV
  hbar      = 0.6582119569 eV*fs
  k_B       = 8.617333262e-5 eV/K
  a0        = 0.529177210903 Angstrom (Bohr radius)
  e/(4 pi eps0) = 14.399645478425 V*Angstrom
  2 pi a0 e = 2 pi * a0 * e/(4 pi eps0)  (V*Angstrom^2), the prefactor of projected potentials
"""
import math

import numpy as np

HC_EV_A = 12398.419843320026
M0C2_EV = 510998.95
HBAR_EV_FS = 0.6582119569
KB_EV_K = 8.617333262e-5
A0_A = 0.529177210903
E_4PIEPS0_V_A = 14.399645478425
TWO_PI_A0_E = 2.0 * math.pi * A0_A * E_4PIEPS0_V_A


def wavelength(energy_ev):
    """Relativistic electron wavelength lambda = hc / sqrt(E (2 m0c^2 + E)) in Angstrom."""
    e = float(energy_ev)
    return HC_EV_A / math.sqrt(e * (2.0 * M0C2_EV + e))


def interaction_parameter(energy_ev):
    """sigma = (2 pi / (lambda E)) (m0c^2 + E) / (2 m0c^2 + E) in rad / (V*Angstrom)."""
    e = float(energy_ev)
    return (2.0 * math.pi / (wavelength(e) * e)) * (M0C2_EV + e) / (2.0 * M0C2_EV + e)


def energy_axis(n_e, dt_fs):
    """Energy of each bin after the time-to-energy DFT, ascending (fftshifted), in eV.

    A segment of n_e snapshots spaced dt lasts t_tot = n_e dt, so the bin width is
    E_min = 2 pi hbar / t_tot and the largest representable energy is E_max = pi hbar / dt
    (first step of the two-step procedure).  Bin j of the ascending axis holds
    E = (j - n_e//2) * E_min; positive E is an energy loss (E = E_m - E_n in the spectral sum).
    """
    kp = np.arange(n_e) - n_e // 2
    return 2.0 * math.pi * HBAR_EV_FS * kp / (n_e * dt_fs)


def e_min(n_e, dt_fs):
    """Lowest non-zero energy 2 pi hbar / (n_e dt) in eV."""
    return 2.0 * math.pi * HBAR_EV_FS / (n_e * dt_fs)


def e_max(dt_fs):
    """Nyquist energy pi hbar / dt in eV."""
    return math.pi * HBAR_EV_FS / dt_fs


def nyquist_thz(dt_fs):
    """Nyquist frequency 1 / (2 dt) in THz."""
    return 1.0 / (2.0 * dt_fs * 1e-15) / 1e12


def n_segments(n_snap, n_e, hop):
    """Number of complete segments of n_e consecutive snapshots offset by hop (tail dropped)."""
    if n_e > n_snap:
        return 0
    return (n_snap - n_e) // hop + 1


def kubo_factor(energy_ev, temperature_k):
    """Detailed-balance factor beta E / (1 - exp(-beta E)) relating the Kubo-transformed and the
    quantum correlation spectra (equation relating c(E) and c~(E)).  Its value at E = 0 is 1 (the
    limit); near zero the series 1 + x/2 + x^2/12 avoids 0/0."""
    beta = 1.0 / (KB_EV_K * float(temperature_k))
    x = beta * np.asarray(energy_ev, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-4
    out[small] = 1.0 + x[small] / 2.0 + x[small] ** 2 / 12.0
    xs = x[~small]
    out[~small] = xs / (-np.expm1(-xs))
    return out
