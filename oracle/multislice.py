"""Multislice propagation of the auxiliary beam wave through one configuration (oracle, complex128).

The paper propagates the beam through every snapshot of the trajectory with a standard multislice
method and stacks the exit waves phi(q, t) into a three-dimensional dataset (second step of the
procedure; the QEP background introduces phi(q, tau) as the Fourier transform of phi(r, tau)).
Textbook multislice in the convention of the paraxial equation
d psi/dz = (i lambda / 4 pi) laplacian psi + i sigma V psi:

  psi_{s+1} = F^-1 [ M(k) P_s(k) F [ t_s(r) psi_s(r) ] ]
  t_s(r)    = exp(i sigma V_s(r))                      (transmission)
  P_s(k)    = exp(-i pi lambda dz_s (kx^2 + ky^2))       (Fresnel propagator)

with F the unnormalised DFT exp(-2 pi i k.r) and F^-1 = conj(F)/(Nx Ny).  The wave is propagated
after the last slice too, and the exit wave is phi(q) = F[psi_S] / sqrt(Nx Ny), so that
sum_q |phi(q)|^2 = sum_r |psi_S(r)|^2.

Initial waves: a plane wave psi_0 = 1/sqrt(Nx Ny), or a STEM probe
  psi_0(k) proportional to A(k) exp(-i chi(k)) exp(-2 pi i k . r_p),
  A(k) = 1 when (lambda^2) (kx^2 + ky^2) <= alpha^2 (float64), chi = pi lambda df k^2 + pi Cs lambda^3 k^4 / 2,
normalised to sum_r |psi_0(r)|^2 = 1.  Sign reading of the defocus: a probe at defocus df is the
in-focus probe propagated forward by df in vacuum with the propagator above (its crossover lies df
before the entrance plane); chi in terms of the angle theta = lambda |k| is the textbook
(2 pi / lambda) (Cs theta^4 / 4 + df theta^2 / 2).  (The paper's Fe run defines its probe only by the
convergence semi-angle.)
"""
import math

import numpy as np

from .dft import dft2, idft2
from .physics import wavelength, interaction_parameter
from .potential import bandlimit_mask, k_vectors


def propagator(spec, energy_ev, dz):
    """M(k) exp(-i pi lambda dz |k|^2), complex128 [ny][nx]."""
    lam = wavelength(energy_ev)
    kx, ky = k_vectors(spec.nx, spec.ny, spec.lx, spec.ly)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    mask = bandlimit_mask(spec.nx, spec.ny, spec.lx, spec.ly, spec.bandlimit)
    return mask * np.exp(-1j * math.pi * lam * dz * k2)


def plane_wave(spec):
    n = spec.nx * spec.ny
    return np.full((spec.ny, spec.nx), 1.0 / math.sqrt(n), dtype=np.complex128)


def probe_wave(spec, beam, pos_xy):
    """STEM probe centred at pos_xy (Angstrom), normalised to unit total intensity."""
    lam = wavelength(beam.energy_ev)
    kx, ky = k_vectors(spec.nx, spec.ny, spec.lx, spec.ly)
    k2 = ky[:, None] * ky[:, None] + kx[None, :] * kx[None, :]
    aperture = ((lam * lam) * k2 <= beam.alpha_rad * beam.alpha_rad).astype(np.float64)
    chi = math.pi * lam * beam.defocus_a * k2 + 0.5 * math.pi * beam.cs_a * lam ** 3 * k2 ** 2
    shift = np.exp(-2j * math.pi * (kx[None, :] * pos_xy[0] + ky[:, None] * pos_xy[1]))
    a = aperture * np.exp(-1j * chi) * shift
    psi = idft2(a)                                # sum_k a(k) exp(+2 pi i k.r)
    return psi / math.sqrt(np.sum(np.abs(psi) ** 2))


def initial_waves(spec, beam):
    """psi_0 for every probe position: complex128 [P][ny][nx]."""
    if not beam.probe:
        return plane_wave(spec)[None]
    return np.stack([probe_wave(spec, beam, p) for p in beam.probe_xy])


def transmission(V, sigma):
    return np.exp(1j * sigma * V)


def propagate(psi0, V, spec, energy_ev, keep_states=False):
    """Run the multislice through the S slices of one configuration.

    psi0: [ny][nx] complex; V: [S][ny][nx] real (V*Angstrom).  Returns the exit wave phi(q)
    [ny][nx] in DFT storage order, and with keep_states the pre-transmission real-space waves
    psi_s for s = 0..S-1 ([S][ny][nx])."""
    sigma = interaction_parameter(energy_ev)
    n = spec.nx * spec.ny
    psi = np.array(psi0, dtype=np.complex128)
    states = []
    S = V.shape[0]
    for s in range(S):
        if keep_states:
            states.append(psi.copy())
        prop = propagator(spec, energy_ev, spec.dz[s])
        u = transmission(V[s], sigma) * psi
        if s < S - 1:
            psi = idft2(prop * dft2(u)) / n
        else:
            phi = prop * dft2(u) / math.sqrt(n)
    if keep_states:
        return phi, np.stack(states)
    return phi


def exit_waves(V, spec, beam):
    """phi(q, t) for every snapshot and probe position: complex128 [T][P][ny][nx]."""
    psi0 = initial_waves(spec, beam)
    T = V.shape[0]
    out = np.empty((T, psi0.shape[0], spec.ny, spec.nx), dtype=np.complex128)
    for t in range(T):
        for p in range(psi0.shape[0]):
            out[t, p] = propagate(psi0[p], V[t], spec, beam.energy_ev)
    return out
