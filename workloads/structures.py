"""Equilibrium crystal structures for the synthetic workloads.

All cells are orthorhombic and periodic in x and y; the beam travels along +z.  Atomic planes
normal to z are shifted by half the plane spacing so that, when the slice thickness equals the
plane spacing (or a multiple of it), every plane sits strictly inside one slice and thermal
vibrations (RMS 0.07 Angstrom) never carry an atom across a slice boundary.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Structure:
    positions: np.ndarray      # float64 [N][3] equilibrium positions, Angstrom
    species: np.ndarray        # int32 [N] index into `species_names`
    species_names: tuple
    cell: tuple                # (Lx, Ly, Lz) Angstrom
    lattice_a: float           # length used by the synthetic dispersion relation
    plane_spacing: float       # distance between equilibrium atomic planes along z


def _tile(basis_frac, basis_species, cell_abc, reps):
    nx, ny, nz = reps
    ax, ay, az = cell_abc
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    origins = np.stack([ii.ravel() * ax, jj.ravel() * ay, kk.ravel() * az], axis=1)   # [C][3]
    frac = np.asarray(basis_frac, dtype=np.float64) * np.array([ax, ay, az])
    pos = (origins[:, None, :] + frac[None, :, :]).reshape(-1, 3)
    spc = np.tile(np.asarray(basis_species, dtype=np.int32), origins.shape[0])
    # order atoms by z plane, then y, then x: slices then hold contiguous index ranges
    order = np.lexsort((pos[:, 0], pos[:, 1], np.round(pos[:, 2], 6)))
    return pos[order], spc[order]


def fcc_cubic(a=4.0, reps=(4, 4, 4)):
    """Face-centred cubic, one species "A"; planes every a/2 along z."""
    basis = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    pos, spc = _tile(basis, [0, 0, 0, 0], (a, a, a), reps)
    pos[:, 2] += a / 4.0
    return Structure(pos, spc, ("A",), (a * reps[0], a * reps[1], a * reps[2]), a, a / 2.0)


def rocksalt(a=4.0, reps=(10, 10, 20)):
    """Rocksalt-like A/B crystal: A on fcc sites, B shifted by (a/2, 0, 0); planes every a/2."""
    fcc = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    basis = fcc + [((x + 0.5) % 1.0, y, z) for (x, y, z) in fcc]
    pos, spc = _tile(basis, [0] * 4 + [1] * 4, (a, a, a), reps)
    pos[:, 2] += a / 4.0
    return Structure(pos, spc, ("A", "B"), (a * reps[0], a * reps[1], a * reps[2]), a, a / 2.0)


def hexagonal_bn_like(a=2.50, c=6.66, reps=(16, 9, 10)):
    """B/N-like honeycomb layers in AA' stacking, orthogonal cell a x sqrt(3)a x c.

    Two layers per c; the second layer has the two species swapped.  The in-plane lattice
    parameter 2.50 Angstrom is the hexagonal one (the bond length is a/sqrt(3) = 1.443 Angstrom).
    """
    b = np.sqrt(3.0) * a
    layer = [(0.0, 0.0), (0.5, 0.5), (0.5, 1.0 / 6.0), (0.0, 2.0 / 3.0)]
    basis, spc = [], []
    for x, y in layer[:2]:
        basis.append((x, y, 0.0)); spc.append(0)
    for x, y in layer[2:]:
        basis.append((x, y, 0.0)); spc.append(1)
    for x, y in layer[:2]:
        basis.append((x, y, 0.5)); spc.append(1)
    for x, y in layer[2:]:
        basis.append((x, y, 0.5)); spc.append(0)
    pos, s = _tile(basis, spc, (a, b, c), reps)
    pos[:, 2] += c / 4.0
    return Structure(pos, s, ("BN-B", "BN-N"), (a * reps[0], b * reps[1], c * reps[2]), a, c / 2.0)


def diamond_cubic(a=5.4773, reps=(7, 7, 92)):
    """Diamond-structure crystal of one species "A" (silicon-like): two fcc lattices offset by
    (a/4, a/4, a/4).  Atomic planes every a/4 along z, shifted by a/16 so that they sit inside a
    slice for slice thicknesses of a/4 or a/8 (the paper's Si runs use 8 slices per cubic cell)."""
    fcc = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    basis = fcc + [(x + 0.25, y + 0.25, z + 0.25) for (x, y, z) in fcc]
    pos, spc = _tile(basis, [0] * 8, (a, a, a), reps)
    pos[:, 2] += a / 16.0
    return Structure(pos, spc, ("A",), (a * reps[0], a * reps[1], a * reps[2]), a, a / 4.0)


def bcc_cubic(a=2.87, reps=(20, 20, 10)):
    """Body-centred cubic crystal of one species "B" (iron-like); planes every a/2 along z,
    shifted by a/8 (inside a slice for thicknesses a/2 down to a/4, and for the thin slices of
    multislice runs whose planes are resolved by several slices)."""
    basis = [(0, 0, 0), (0.5, 0.5, 0.5)]
    pos, spc = _tile(basis, [0, 0], (a, a, a), reps)
    pos[:, 2] += a / 8.0
    return Structure(pos, spc, ("B",), (a * reps[0], a * reps[1], a * reps[2]), a, a / 2.0)
