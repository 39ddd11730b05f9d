"""Pins of the oracle's analysis outputs: the energy-integrated patterns against the direct QEP
average (Parseval), a static lattice, the detailed-balance ratio of a two-line spectrum, the
relative-difference profile and the bilinear path cut (exact on pixels and on linear fields)."""
import math

import numpy as np
import pytest

from oracle import analysis as an
from oracle.physics import HBAR_EV_FS, kubo_factor


def _rand_stack(T, P, ny, nx, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(T, P, ny, nx)) + 1j * rng.normal(size=(T, P, ny, nx))


def test_energy_integral_of_ctilde_is_the_qep_pattern_of_the_same_snapshots():
    x = _rand_stack(24, 2, 6, 8, 0)
    n_e = 8
    ct, _ = an.energy_integrals_from_exit(x, n_e, n_e, 5.0, 300.0, 6, 8)
    # QEP from the definition: mean |phi|^2 over the 24 snapshots and both positions, normalised,
    # centred with the library's fftshift
    I = np.sum(np.abs(x) ** 2, axis=(0, 1))
    ref = np.fft.fftshift(I / I.sum())
    np.testing.assert_allclose(ct, ref, rtol=1e-12)
    np.testing.assert_allclose(an.qep_pattern(x, range(24), 6, 8), ref, rtol=1e-12)


def test_qep_subset_and_crop():
    x = _rand_stack(10, 1, 8, 8, 1)
    sub = [1, 4, 7]
    I = np.sum(np.abs(x[sub]) ** 2, axis=(0, 1))
    full = np.fft.fftshift(I / I.sum())
    np.testing.assert_allclose(an.qep_pattern(x, sub, 5, 3), full[4 - 2:4 + 3, 4 - 1:4 + 2],
                               rtol=1e-12)


def test_static_lattice_patterns_agree():
    rng = np.random.default_rng(2)
    phi = rng.normal(size=(1, 2, 4, 6)) + 1j * rng.normal(size=(1, 2, 4, 6))
    x = np.repeat(phi, 16, axis=0)
    ct, c = an.energy_integrals_from_exit(x, 16, 16, 5.0, 300.0, 4, 6)
    qep = an.qep_pattern(x, range(16), 4, 6)
    np.testing.assert_allclose(ct, qep, rtol=1e-12)
    np.testing.assert_allclose(c, qep, rtol=1e-12)


def test_detailed_balance_ratio_of_a_two_line_spectrum():
    # pixel a oscillates at E0 > 0 (all its weight in the loss bin k0), pixel b is static (E = 0):
    # c(a)/c(b) = K(E0) * c~(a)/c~(b)
    n_e, dt, k0, T = 32, 5.0, 3, 300.0
    e0 = 2 * math.pi * HBAR_EV_FS * k0 / (n_e * dt)
    t = np.arange(n_e)
    x = np.zeros((n_e, 1, 2, 2), dtype=complex)
    x[:, 0, 0, 1] = 0.7 * np.exp(2j * math.pi * k0 * t / n_e)
    x[:, 0, 1, 0] = 0.4
    ct, c = an.energy_integrals_from_exit(x, n_e, n_e, dt, T, 2, 2)
    # centred layout of a 2 x 2 grid: storage (0, 1) -> (1, 0), storage (1, 0) -> (0, 1)
    ra, rb = (1, 0), (0, 1)
    assert c[ra] / c[rb] == pytest.approx(kubo_factor(e0, T) * ct[ra] / ct[rb], rel=1e-12)
    assert ct[ra] / ct[rb] == pytest.approx(0.49 / 0.16, rel=1e-12)


def test_relative_difference_row():
    A = np.array([[9.0, 9.0, 9.0], [1.0, 3.0, 0.0], [5.0, 5.0, 5.0]])
    B = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 0.0], [5.0, 5.0, 5.0]])
    np.testing.assert_allclose(an.relative_difference_row(A, B), [0.0, 0.5, 0.0])
    np.testing.assert_allclose(an.relative_difference_row(B, A), [0.0, -0.5, 0.0])
    np.testing.assert_allclose(an.relative_difference_row(A, A), [0.0, 0.0, 0.0])


def test_path_points_polyline():
    v = [(0.0, 0.0), (1.0, 0.0), (1.0, 2.0)]
    p = an.path_points(v, 4)
    assert p.shape == (9, 2)
    np.testing.assert_allclose(p[0], v[0])
    np.testing.assert_allclose(p[4], v[1])
    np.testing.assert_allclose(p[-1], v[2])
    np.testing.assert_allclose(p[6], (1.0, 1.0))


def test_path_cut_exact_on_pixels_and_linear_fields():
    n_e, nqy, nqx, lx, ly = 3, 9, 12, 20.0, 15.0
    rng = np.random.default_rng(4)
    S = rng.uniform(size=(n_e, nqy, nqx))
    # q on pixel centres: the pixel's value
    pts = [((ix - nqx // 2) / lx, (iy - nqy // 2) / ly) for iy, ix in ((0, 0), (4, 6), (8, 11))]
    got = an.path_cut(S, lx, ly, pts)
    for n, (iy, ix) in enumerate(((0, 0), (4, 6), (8, 11))):
        np.testing.assert_allclose(got[:, n], S[:, iy, ix], rtol=1e-13)
    # a field linear in the pixel coordinates is reproduced between pixels
    jj, ii = np.meshgrid(np.arange(nqy), np.arange(nqx), indexing="ij")
    L = np.stack([2.0 + 0.5 * ii - 0.25 * jj, -1.0 + 0.1 * ii + 0.3 * jj, 0.7 * ii])
    pts = an.path_points([(-0.2, -0.2), (0.2, 0.15)], 7)
    got = an.path_cut(L, lx, ly, pts)
    for n, (qx, qy) in enumerate(pts):
        u, v = qx * lx + nqx // 2, qy * ly + nqy // 2
        np.testing.assert_allclose(got[:, n], [2.0 + 0.5 * u - 0.25 * v, -1.0 + 0.1 * u + 0.3 * v,
                                               0.7 * u], rtol=1e-12)
    # far outside the map: zero
    assert np.all(an.path_cut(S, lx, ly, [(5.0, 5.0)]) == 0)
