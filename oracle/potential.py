"""Slice binning and projected slice potentials (oracle, FP64).

The paper obtains the auxiliary wave phi(q, tau) of each configuration tau "by a standard
multislice method" and leaves the potentials to its multislice programs (QEP background; second
step of the procedure).  The textbook construction used here:

* Slices are half-open intervals [z_s, z_{s+1}) with z_0 = z0 and z_{s+1} = z_s + dz_s (summed in
  float64 in slice order).  An atom belongs to the slice whose interval holds its z; atoms
  outside [z_0, z_S) belong to no slice and are dropped.
* The electron form factor of species Z is f_Z(q) = sum_i a_i/(q^2+b_i) + sum_i c_i exp(-d_i q^2).
* On the periodic cell Lx x Ly the Fourier coefficients of the projected potential of slice s are
      V_s(k) = (2 pi a0 e / (Lx Ly)) M(k) sum_{j in s} f_{Z_j}(|k|) exp(-2 pi i k . r_j)
  with k = (m/Lx, n/Ly) for the signed DFT indices m, n, and the real-space map on the grid is
      V_s(r) = Re sum_k V_s(k) exp(+2 pi i k . r).
* The band limit M(k) = 1 when kx^2 + ky^2 < (f k_N)^2 with k_N = min(Nx/(2Lx), Ny/(2Ly)); all
  quantities in float64, kx = m/Lx computed as one division.  f <= 0 disables the band limit.
"""
import numpy as np

from .dft import fftfreq_index, idft2
from .physics import TWO_PI_A0_E


def slice_boundaries(z0, dz):
    """z_0 .. z_S accumulated left to right in float64."""
    b = np.empty(len(dz) + 1, dtype=np.float64)
    b[0] = float(z0)
    for s, d in enumerate(dz):
        b[s + 1] = b[s] + float(d)
    return b


def bin_atoms(z, boundaries):
    """Slice index of each atom (int64), -1 for atoms outside [z_0, z_S).

    z_s <= z < z_{s+1} is decided in float64 (float32 inputs convert exactly)."""
    z = np.asarray(z).astype(np.float64)
    s = np.searchsorted(boundaries, z, side="right") - 1
    s[(z < boundaries[0]) | (z >= boundaries[-1])] = -1
    return s


def form_factor(ff_row, q):
    """f(q) = sum_i a_i/(q^2+b_i) + c_i exp(-d_i q^2); ff_row = a1,b1,a2,b2,a3,b3,c1,d1,c2,d2,c3,d3."""
    q2 = np.asarray(q, dtype=np.float64) ** 2
    a, b = ff_row[0:6:2], ff_row[1:6:2]
    c, d = ff_row[6:12:2], ff_row[7:12:2]
    out = np.zeros_like(q2)
    for i in range(3):
        if a[i] != 0.0:
            out += a[i] / (q2 + b[i])
        if c[i] != 0.0:
            out += c[i] * np.exp(-d[i] * q2)
    return out


def k_vectors(nx, ny, lx, ly):
    """kx[m] = m/Lx, ky[n] = n/Ly for the signed DFT indices in storage order (1/Angstrom)."""
    kx = fftfreq_index(nx) / float(lx)
    ky = fftfreq_index(ny) / float(ly)
    return kx, ky


def bandlimit_mask(nx, ny, lx, ly, fraction):
    """M(k) as float64 [ny][nx] (1 inside the band limit, 0 outside)."""
    if fraction <= 0.0:
        return np.ones((ny, nx))
    kx, ky = k_vectors(nx, ny, lx, ly)
    kn = min(nx / (2.0 * lx), ny / (2.0 * ly))
    kmax = fraction * kn
    k2 = ky[:, None] * ky[:, None] + kx[None, :] * kx[None, :]
    return (k2 < kmax * kmax).astype(np.float64)


def slice_potential_k(xy, species, ff, nx, ny, lx, ly, mask):
    """V_s(k) [ny][nx] complex128 for the atoms of one slice (xy [A][2] Angstrom).

    The phase exp(-2 pi i (kx x + ky y)) is the product of an x factor and a y factor, so the
    structure factor of each species is the matrix product Ey^T Ex of the per-atom phase tables;
    this is the same sum as the direct double loop, evaluated with a BLAS product."""
    xy = np.asarray(xy, dtype=np.float64)
    kx, ky = k_vectors(nx, ny, lx, ly)
    kabs = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    vk = np.zeros((ny, nx), dtype=np.complex128)
    for z in range(ff.shape[0]):
        sel = species == z
        if not np.any(sel):
            continue
        ex = np.exp(-2j * np.pi * np.outer(xy[sel, 0], kx))        # [A][nx]
        ey = np.exp(-2j * np.pi * np.outer(xy[sel, 1], ky))        # [A][ny]
        sf = ey.T @ ex                                             # [ny][nx]
        vk += form_factor(ff[z], kabs) * sf
    return (TWO_PI_A0_E / (lx * ly)) * mask * vk


def slice_potential_k_direct(xy, species, ff, nx, ny, lx, ly, mask):
    """The same V_s(k) as a literal loop over k points and atoms (small cases only)."""
    kx, ky = k_vectors(nx, ny, lx, ly)
    vk = np.zeros((ny, nx), dtype=np.complex128)
    for n in range(ny):
        for m in range(nx):
            if mask[n, m] == 0.0:
                continue
            kabs = np.sqrt(kx[m] ** 2 + ky[n] ** 2)
            acc = 0j
            for j in range(len(species)):
                f = form_factor(ff[species[j]], np.array([kabs]))[0]
                acc += f * np.exp(-2j * np.pi * (kx[m] * xy[j][0] + ky[n] * xy[j][1]))
            vk[n, m] = acc
    return (TWO_PI_A0_E / (lx * ly)) * vk


def slice_potential(xy, species, ff, nx, ny, lx, ly, mask):
    """V_s(r_n) on the grid, float64 [ny][nx], in V*Angstrom."""
    return idft2(slice_potential_k(xy, species, ff, nx, ny, lx, ly, mask)).real


def potentials(positions, species, ff, spec):
    """V[T][S][ny][nx] float64 for every snapshot and slice, plus the slice index of every atom.

    `spec` provides nx, ny, lx, ly, dz (array), z0 and bandlimit.  Positions are used at the
    precision they come in (the GPU library takes float32 positions; pass the same array)."""
    pos = np.asarray(positions).astype(np.float64)
    T = pos.shape[0]
    S = len(spec.dz)
    bnd = slice_boundaries(spec.z0, spec.dz)
    mask = bandlimit_mask(spec.nx, spec.ny, spec.lx, spec.ly, spec.bandlimit)
    V = np.zeros((T, S, spec.ny, spec.nx))
    bins = np.empty((T, pos.shape[1]), dtype=np.int64)
    for t in range(T):
        bins[t] = bin_atoms(pos[t, :, 2], bnd)
        for s in range(S):
            sel = bins[t] == s
            V[t, s] = slice_potential(pos[t, sel, :2], species[sel], ff, spec.nx, spec.ny,
                                      spec.lx, spec.ly, mask)
    return V, bins
