"""Analysis outputs of the method's spectra (oracle, FP64; test infrastructure only).

Paper passages followed (the Si and hBN results paragraphs, Figs. 1 and 2):
* Diffraction patterns from the method: the energy integral of the spectrum at each q, both of the
  classical time-average c~(q, E) (before the detailed-balance correction) and of the corrected
  c(q, E).  Each map is normalised to unit total over the full q grid, so that patterns from
  different methods compare as fractional intensities.
* The standard QEP (quantum excitation of phonons) pattern: the diffraction intensity |phi(q, tau)|^2
  averaged incoherently over a set of snapshots (evenly spaced ones, or all of them) and over probe
  positions, normalised the same way.  By Parseval's theorem the energy integral of c~ over
  non-overlapping segments equals the QEP pattern of the same snapshots (a pin in the tests).
* Line profiles: the relative difference (A - B) / (A + B) of two patterns along theta_y = 0, the
  q_y = 0 row of the centred maps.
* Dispersion plots: S(q, E) along a polyline through high-symmetry points of the q plane, sampled
  bilinearly on the centred pixel grid q = m / L (pixels outside the map count as zero).

All maps use the layout of the spectrum output: centred q (index i holds the signed frequency
i - nq // 2), cropped to nqy x nqx; energies ascending.
"""
import numpy as np

from .spectrum import kubo_table_dft_order, segment_periodogram, shift_and_crop


def _centred_crop(full_map, nqy, nqx):
    """[ny][nx] map in DFT storage order -> centred crop [nqy][nqx]."""
    return shift_and_crop(full_map[None], nqy, nqx)[0]


def energy_integrals(P_dft, K_dft, nqy, nqx):
    """From a periodogram P [n_e][ny][nx] (DFT order) and the Kubo factors of its bins:
    (c~ map, c map), each the sum over energies divided by its total over the full q grid."""
    ct = np.sum(P_dft, axis=0)
    c = np.sum(K_dft[:, None, None] * P_dft, axis=0)
    return _centred_crop(ct / np.sum(ct), nqy, nqx), _centred_crop(c / np.sum(c), nqy, nqx)


def energy_integrals_from_exit(exit_stack, n_e, hop, dt_fs, temperature_k, nqy, nqx):
    """Energy-integrated maps of the spectrum of an exit-wave stack [T][P][ny][nx]."""
    P = segment_periodogram(exit_stack, n_e, hop)
    return energy_integrals(P, kubo_table_dft_order(n_e, dt_fs, temperature_k), nqy, nqx)


def qep_pattern(exit_stack, t_index, nqy, nqx):
    """Mean over the snapshots t_index and all probe positions of |phi(q)|^2, normalised to unit
    total over the full grid, centred and cropped."""
    sel = exit_stack[np.asarray(t_index)]
    I = np.sum(np.abs(sel) ** 2, axis=(0, 1))
    return _centred_crop(I / np.sum(I), nqy, nqx)


def relative_difference_row(A, B):
    """(A - B) / (A + B) along the q_y = 0 row (index nqy // 2) of two centred maps; 0 where
    A + B = 0."""
    a = A[A.shape[0] // 2].astype(np.float64)
    b = B[B.shape[0] // 2].astype(np.float64)
    s = a + b
    out = np.zeros_like(s)
    nz = s != 0
    out[nz] = (a[nz] - b[nz]) / s[nz]
    return out


def path_points(vertices, n_per_seg):
    """Points along the polyline through vertices [(qx, qy)] (1/Angstrom): n_per_seg points per
    segment starting at its first vertex, and the last vertex once at the end."""
    v = np.asarray(vertices, dtype=np.float64)
    pts = []
    for s in range(len(v) - 1):
        for j in range(n_per_seg):
            pts.append(v[s] + (j / n_per_seg) * (v[s + 1] - v[s]))
    pts.append(v[-1])
    return np.array(pts)


def path_cut(S, lx, ly, points):
    """S [n_e][nqy][nqx] (centred q) sampled bilinearly at q points [n][2] (1/Angstrom) ->
    [n_e][n].  The fractional pixel position of q is (qx lx + nqx // 2, qy ly + nqy // 2)."""
    n_e, nqy, nqx = S.shape
    out = np.zeros((n_e, len(points)))

    def pix(iy, ix):
        if 0 <= iy < nqy and 0 <= ix < nqx:
            return S[:, iy, ix].astype(np.float64)
        return np.zeros(n_e)

    for n, (qx, qy) in enumerate(points):
        u = qx * lx + nqx // 2
        v = qy * ly + nqy // 2
        i0, j0 = int(np.floor(u)), int(np.floor(v))
        fx, fy = u - i0, v - j0
        out[:, n] = ((1 - fx) * (1 - fy) * pix(j0, i0) + fx * (1 - fy) * pix(j0, i0 + 1) +
                     (1 - fx) * fy * pix(j0 + 1, i0) + fx * fy * pix(j0 + 1, i0 + 1))
    return out
