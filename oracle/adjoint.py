"""Hand-written FP64 adjoints of the spectrum, the multislice and the slice potentials (oracle).

Gradient convention (the one PyTorch uses): for a real loss L and a complex variable z the
gradient is G_z = dL/dRe z + i dL/dIm z (= 2 dL/d conj(z)); for a linear map z' = A z this gives
G_z = A^H G_z'.  For real variables it is the ordinary derivative.

Chain (all derived from the forward definitions in `spectrum`, `multislice` and `potential`):

1. Normalisation I = K P / Z with Z = sum K P over the full grid:
       dL/dP = (K / Z) (g - sum(g I)),  g = dL/dI (zero outside the cropped q window).
2. Segment periodogram P = (1/G) sum_g sum_p |Phi_g|^2, Phi_g(k) = sum_t phi(t_g + t) e^{-2 pi i k t/n_e}:
       G_phi(t_g + t) += (2/G) sum_k dL/dP(k) Phi_g(k) e^{+2 pi i k t / n_e}.
3. Multislice, u_s = t_s psi_s, psi_{s+1} = F^-1 D_s F u_s, phi = D_{S-1} F u_{S-1} / sqrt(N):
       chi_{S-1} = F^-1[conj(D_{S-1}) G_phi] * sqrt(N)  (= idft(conj(D) G_phi)/sqrt(N) unnormalised),
       dL/dV_s = -sigma Im(conj(chi_s) t_s psi_s),
       G_psi_s = conj(t_s) chi_s,  chi_{s-1} = F^-1[conj(D_{s-1}) F G_psi_s].
4. Potential V_s(r) = Re sum_k V_s(k) e^{2 pi i k.r}:
       dL/dx_j = Re sum_k conj(Ghat(k)) C M(k) f_Zj(|k|) (-2 pi i kx) e^{-2 pi i k.r_j},  Ghat = F[dL/dV_s],
   and likewise for y_j; dL/dz_j = 0 because slice membership is piecewise constant in z.
"""
import math

import numpy as np

from .dft import dft2, idft2, dft_axis
from .multislice import propagator, transmission, propagate, initial_waves
from .physics import interaction_parameter, n_segments, TWO_PI_A0_E
from .potential import (bandlimit_mask, form_factor, k_vectors, slice_boundaries, bin_atoms,
                        potentials)
from .spectrum import kubo_table_dft_order, segment_periodogram


def _uncrop(g_s, n_e, ny, nx):
    nqy, nqx = g_s.shape[1:]
    e_idx = (np.arange(n_e) - n_e // 2) % n_e
    y_idx = (np.arange(nqy) - nqy // 2) % ny
    x_idx = (np.arange(nqx) - nqx // 2) % nx
    full = np.zeros((n_e, ny, nx))
    full[np.ix_(e_idx, y_idx, x_idx)] = g_s
    return full


def spectrum_backward(exit_stack, g_s, n_e, hop, dt_fs, temperature_k):
    """G_phi [T][P][ny][nx] (PyTorch convention) from g = dL/dS on the output grid [n_e][nqy][nqx]."""
    T = exit_stack.shape[0]
    ny, nx = exit_stack.shape[-2:]
    G = n_segments(T, n_e, hop)
    P = segment_periodogram(exit_stack, n_e, hop)
    K = kubo_table_dft_order(n_e, dt_fs, temperature_k)
    Z = float(np.sum(K[:, None, None] * P))
    I_full = K[:, None, None] * P / Z
    g = _uncrop(g_s, n_e, ny, nx)
    gP = (K[:, None, None] / Z) * (g - np.sum(g * I_full))
    out = np.zeros(exit_stack.shape, dtype=np.complex128)
    for s in range(G):
        seg = exit_stack[s * hop: s * hop + n_e]
        phi_k = dft_axis(seg, axis=0)
        back = dft_axis(gP[:, None] * phi_k, axis=0, inverse=True)
        out[s * hop: s * hop + n_e] += (2.0 / G) * back
    return out


def multislice_adjoint(psi0, V, spec, energy_ev, g_phi, return_g_psi0=False):
    """dL/dV_s [S][ny][nx] for one wave, given G_phi [ny][nx] of its exit wave.

    With return_g_psi0 the adjoint wave at the entrance surface, G_psi0 = A^H G_phi for the
    linear map A: psi_0 -> phi at fixed V, is returned as well."""
    sigma = interaction_parameter(energy_ev)
    n = spec.nx * spec.ny
    _, states = propagate(psi0, V, spec, energy_ev, keep_states=True)
    S = V.shape[0]
    gV = np.zeros(V.shape)
    chi = idft2(np.conj(propagator(spec, energy_ev, spec.dz[S - 1])) * g_phi) / math.sqrt(n)
    for s in range(S - 1, -1, -1):
        t = transmission(V[s], sigma)
        gV[s] = -sigma * np.imag(np.conj(chi) * t * states[s])
        g_psi = np.conj(t) * chi
        if s > 0:
            chi = idft2(np.conj(propagator(spec, energy_ev, spec.dz[s - 1])) * dft2(g_psi)) / n
    if return_g_psi0:
        return gV, g_psi
    return gV


def position_gradient(gV, xyz, species, ff, spec):
    """dL/d(x_j, y_j) [N][2] for one snapshot from dL/dV [S][ny][nx]."""
    xyz = np.asarray(xyz).astype(np.float64)
    bins = bin_atoms(xyz[:, 2], slice_boundaries(spec.z0, spec.dz))
    kx, ky = k_vectors(spec.nx, spec.ny, spec.lx, spec.ly)
    kabs = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    mask = bandlimit_mask(spec.nx, spec.ny, spec.lx, spec.ly, spec.bandlimit)
    c = TWO_PI_A0_E / (spec.lx * spec.ly)
    out = np.zeros((xyz.shape[0], 2))
    for s in range(gV.shape[0]):
        ghat = dft2(gV[s])
        for z in range(ff.shape[0]):
            sel = np.nonzero((bins == s) & (species == z))[0]
            if sel.size == 0:
                continue
            h = np.conj(ghat) * c * mask * form_factor(ff[z], kabs)          # [ny][nx]
            ex = np.exp(-2j * np.pi * np.outer(xyz[sel, 0], kx))             # [A][nx]
            ey = np.exp(-2j * np.pi * np.outer(xyz[sel, 1], ky))             # [A][ny]
            hx = h * (-2j * np.pi * kx[None, :])
            hy = h * (-2j * np.pi * ky[:, None])
            out[sel, 0] = np.real(np.sum((ey @ hx) * ex, axis=1))
            out[sel, 1] = np.real(np.sum((ey @ hy) * ex, axis=1))
    return out


# ----------------------------------------------------------------------------------------------
# The differentiation workload: loss on energy-filtered diffraction, and its full gradient.

def energy_filter_mask(n_e, dt_fs, e_lo_ev, e_hi_ev):
    """Boolean [n_e] over the ascending energy axis: e_lo <= E <= e_hi."""
    from .physics import energy_axis
    e = energy_axis(n_e, dt_fs)
    return (e >= e_lo_ev) & (e <= e_hi_ev)


def filtered_loss(S, target, emask):
    """L = sum_q (sum_{E in filter} S(q, E) - target(q))^2 and dL/dS."""
    If = np.sum(S[emask], axis=0)
    d = If - target
    g = np.zeros_like(S)
    g[emask] = 2.0 * d[None]
    return float(np.sum(d * d)), g


def forward_all(positions, species, ff, spec, beam, n_e, hop, dt_fs, temperature_k):
    """positions -> (V, exit stack, S, Z)."""
    from .multislice import exit_waves
    from .spectrum import spectrum
    V, _ = potentials(positions, species, ff, spec)
    ex = exit_waves(V, spec, beam)
    S, Z = spectrum(ex, n_e, hop, dt_fs, temperature_k)
    return V, ex, S, Z


def pipeline_gradient(positions, species, ff, spec, beam, n_e, hop, dt_fs, temperature_k,
                      target, emask):
    """Loss and its gradients w.r.t. every V_s(t) and every atom's (x, y) for the filtered loss."""
    V, ex, S, _ = forward_all(positions, species, ff, spec, beam, n_e, hop, dt_fs, temperature_k)
    loss, gS = filtered_loss(S, target, emask)
    g_ex = spectrum_backward(ex, gS, n_e, hop, dt_fs, temperature_k)
    psi0 = initial_waves(spec, beam)
    gV = np.zeros(V.shape)
    for t in range(V.shape[0]):
        for p in range(psi0.shape[0]):
            gV[t] += multislice_adjoint(psi0[p], V[t], spec, beam.energy_ev, g_ex[t, p])
    gxy = np.stack([position_gradient(gV[t], positions[t], species, ff, spec)
                    for t in range(V.shape[0])])
    return dict(loss=loss, V=V, exit=ex, S=S, gS=gS, g_exit=g_ex, gV=gV, gxy=gxy)
