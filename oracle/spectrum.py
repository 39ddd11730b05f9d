"""Time auto-correlation spectrum I(q, E) from the exit-wave stack (oracle, FP64).

Paper passages followed:
* Spectral decomposition: I(q, E) is the time-to-energy Fourier transform, with kernel
  exp(-i E t / hbar), of the auto-correlation <phi^dagger(q, 0) phi(q, t)>; E = E_m - E_n > 0 is a
  loss.  On a segment of n_e snapshots this is the DFT with exp(-2 pi i k t / n_e) of the
  circular auto-correlation sum_t conj(phi(t)) phi(t + tau), which equals |sum_t phi(t)
  exp(-2 pi i k t / n_e)|^2 (convolution theorem; main formula of the method).
* The MD time average yields the Kubo-transformed spectrum; the detailed-balance factor
  beta E / (1 - exp(-beta E)) converts it to the quantum one.
* Fractional intensity: the sum over all q of the grid and all energies (gains and losses) is 1.
* Averaging over segments of one trajectory: segment g covers snapshots g*hop .. g*hop+n_e-1,
  G = floor((T - n_e)/hop) + 1 (a partial tail is dropped).
* Probe positions are summed incoherently before normalising.

Output layout: S[e][iy][ix] with energies ascending (bin e has k' = e - n_e//2) and the q grid
centred (index i holds the signed frequency i - nq//2), cropped to nqy x nqx.
"""
import numpy as np

from .dft import dft_axis, dft_matrix
from .physics import energy_axis, kubo_factor, n_segments


def segment_periodogram(exit_stack, n_e, hop):
    """P(q, k) = (1/G) sum_g sum_p |Phi_g(q, k)|^2 in DFT bin order: float64 [n_e][ny][nx].

    exit_stack: [T][P][ny][nx].  Phi_g is the dense time-DFT of segment g."""
    T = exit_stack.shape[0]
    G = n_segments(T, n_e, hop)
    if G < 1:
        raise ValueError("trajectory shorter than one segment")
    acc = np.zeros((n_e,) + exit_stack.shape[2:], dtype=np.float64)
    for g in range(G):
        seg = exit_stack[g * hop: g * hop + n_e]                 # [n_e][P][ny][nx]
        phi_k = dft_axis(seg, axis=0)                            # exp(-2 pi i k t / n_e)
        acc += np.sum(np.abs(phi_k) ** 2, axis=1)
    return acc / G


def segment_periodogram_bruteforce(exit_stack, n_e, hop):
    """The same P(q, k) from the O(n_e^2) circular auto-correlation followed by its dense DFT:
    c_g(q, tau) = sum_t conj(phi(q, t_g + t)) phi(q, t_g + (t + tau) mod n_e)."""
    T = exit_stack.shape[0]
    G = n_segments(T, n_e, hop)
    f = dft_matrix(n_e)
    acc = np.zeros((n_e,) + exit_stack.shape[2:], dtype=np.float64)
    for g in range(G):
        seg = exit_stack[g * hop: g * hop + n_e]
        corr = np.zeros(seg.shape, dtype=np.complex128)
        for tau in range(n_e):
            for t in range(n_e):
                corr[tau] += np.conj(seg[t]) * seg[(t + tau) % n_e]
        spec = np.tensordot(f, corr, axes=(1, 0))                # sum_tau exp(-2 pi i k tau/n) c(tau)
        acc += np.sum(spec.real, axis=1)
    return acc / G


def shift_and_crop(arr_k, nqy, nqx):
    """Reorder [n_e][ny][nx] from DFT storage order to ascending E and centred, cropped q."""
    n_e, ny, nx = arr_k.shape
    e_idx = (np.arange(n_e) - n_e // 2) % n_e
    y_idx = (np.arange(nqy) - nqy // 2) % ny
    x_idx = (np.arange(nqx) - nqx // 2) % nx
    return arr_k[e_idx][:, y_idx][:, :, x_idx]


def kubo_table_dft_order(n_e, dt_fs, temperature_k):
    """Kubo factor of every DFT bin k (storage order), E_k = 2 pi hbar k' / (n_e dt)."""
    e_asc = energy_axis(n_e, dt_fs)
    k_of_asc = (np.arange(n_e) - n_e // 2) % n_e
    out = np.empty(n_e)
    out[k_of_asc] = kubo_factor(e_asc, temperature_k)
    return out


def spectrum(exit_stack, n_e, hop, dt_fs, temperature_k, nqy=None, nqx=None):
    """I(q, E) normalised to unit total over the full q grid and all energies.

    Returns (S [n_e][nqy][nqx] float64, Z) where Z = sum over the full grid of K * P."""
    ny, nx = exit_stack.shape[-2:]
    nqy = ny if nqy is None else nqy
    nqx = nx if nqx is None else nqx
    P = segment_periodogram(exit_stack, n_e, hop)
    K = kubo_table_dft_order(n_e, dt_fs, temperature_k)
    KP = K[:, None, None] * P
    Z = float(np.sum(KP))
    return shift_and_crop(KP, nqy, nqx) / Z, Z


def kubo_transformed_spectrum(exit_stack, n_e, hop):
    """c~(q, E) before the Kubo correction, unnormalised, E ascending and q centred (full grid)."""
    ny, nx = exit_stack.shape[-2:]
    return shift_and_crop(segment_periodogram(exit_stack, n_e, hop), ny, nx)
