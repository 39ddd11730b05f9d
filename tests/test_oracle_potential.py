"""Pins of the oracle's slice binning and projected potentials against closed forms, exact
identities and a brute-force sum."""
import math
from types import SimpleNamespace

import numpy as np
import pytest
from scipy.special import k0

from oracle import potential as pot
from oracle.physics import TWO_PI_A0_E
from workloads import FORM_FACTORS, form_factor_table


def _periodic_min_dist(rx, ry, x0, y0, lx, ly):
    dx = (rx - x0 + lx / 2) % lx - lx / 2
    dy = (ry - y0 + ly / 2) % ly - ly / 2
    return dx, dy


def test_bin_atoms_half_open_intervals():
    b = pot.slice_boundaries(0.0, [2.0, 2.0, 3.0])
    np.testing.assert_array_equal(b, [0, 2, 4, 7])
    z = np.array([0.0, 1.9999999, 2.0, 3.5, 4.0, 6.9999, 7.0, -1e-6, 100.0], dtype=np.float32)
    np.testing.assert_array_equal(pot.bin_atoms(z, b), [0, 0, 1, 1, 2, 2, -1, -1, -1])


def test_two_pi_a0_e_value():
    # 2 pi a0 e with a0 the Bohr radius and e/(4 pi eps0) = 14.3996 V*Angstrom: 47.8776 V*Angstrom^2
    assert TWO_PI_A0_E == pytest.approx(47.8777, abs=2e-4)


def test_form_factor_at_zero():
    # f(0) = sum a_i/b_i + sum c_i for the invented species A (2.7083 Angstrom)
    f0 = pot.form_factor(FORM_FACTORS["A"], np.array([0.0]))[0]
    assert f0 == pytest.approx(0.30 / 0.15 + 0.20 / 1.5 + 0.05 / 10 + 0.40 + 0.15 + 0.02, rel=1e-14)


def test_k0_integral_identity():
    # sum_r V(r) dx dy = Lx Ly V(k=0) = 2 pi a0 e sum_j f_j(0), exactly, band limit on
    rng = np.random.default_rng(3)
    nx, ny, lx, ly = 32, 16, 9.0, 5.0
    xy = rng.uniform(0, 1, size=(7, 2)) * [lx, ly]
    spc = rng.integers(0, 2, size=7)
    ff = form_factor_table(["A", "B"])
    mask = pot.bandlimit_mask(nx, ny, lx, ly, 2.0 / 3.0)
    V = pot.slice_potential(xy, spc, ff, nx, ny, lx, ly, mask)
    lhs = V.sum() * (lx / nx) * (ly / ny)
    rhs = TWO_PI_A0_E * sum(pot.form_factor(ff[s], np.array([0.0]))[0] for s in spc)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_gaussian_term_matches_closed_form():
    # f = c exp(-d q^2) -> v(r) = 2 pi a0 e c (pi/d) exp(-pi^2 r^2/d); with d k_N^2 = 25 the only
    # error on the grid is the Fourier tail beyond Nyquist (< e^-25)
    nx = ny = 64
    lx = ly = 16.0
    ff = form_factor_table(["gauss-test"])
    c, d = ff[0, 6], ff[0, 7]
    xy = np.array([[7.3, 8.1], [1.2, 15.5]])
    mask = pot.bandlimit_mask(nx, ny, lx, ly, 0.0)
    V = pot.slice_potential(xy, np.array([0, 0]), ff, nx, ny, lx, ly, mask)
    rx = np.arange(nx) * lx / nx
    ry = np.arange(ny) * ly / ny
    RX, RY = np.meshgrid(rx, ry, indexing="xy")
    ref = np.zeros_like(V)
    for x0, y0 in xy:
        for ix in (-1, 0, 1):
            for iy in (-1, 0, 1):
                r2 = (RX - x0 - ix * lx) ** 2 + (RY - y0 - iy * ly) ** 2
                ref += TWO_PI_A0_E * c * (math.pi / d) * np.exp(-math.pi ** 2 * r2 / d)
    assert np.max(np.abs(V - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_lorentzian_term_matches_k0_away_from_core():
    # f = a/(q^2+b) -> v(r) = 2 pi (2 pi a0 e) a K0(2 pi sqrt(b) r); the 1/q^2 tail is cut at
    # Nyquist, so this is a sign-and-scale check at 1..3 Angstrom on a fine grid
    nx = ny = 256
    lx = ly = 16.0
    ff = form_factor_table(["lorentz-test"])
    a, b = ff[0, 0], ff[0, 1]
    x0, y0 = 8.0, 8.0
    mask = pot.bandlimit_mask(nx, ny, lx, ly, 0.0)
    V = pot.slice_potential(np.array([[x0, y0]]), np.array([0]), ff, nx, ny, lx, ly, mask)
    rx = np.arange(nx) * lx / nx
    RX, RY = np.meshgrid(rx, rx, indexing="xy")
    r = np.hypot(RX - x0, RY - y0)
    ref = 2 * math.pi * TWO_PI_A0_E * a * k0(2 * math.pi * math.sqrt(b) * np.maximum(r, 1e-9))
    sel = (r >= 1.0) & (r <= 3.0)
    # the square Nyquist cut leaves Gibbs ripples along the axes: compare in the RMS sense
    rel = np.linalg.norm(V[sel] - ref[sel]) / np.linalg.norm(ref[sel])
    assert rel < 1e-2


def test_integer_pixel_shift_rolls_the_map():
    # moving every atom by (p dx, q dy) rolls V by (q, p) pixels; a wrong phase sign rolls it the
    # other way
    rng = np.random.default_rng(5)
    nx, ny, lx, ly = 32, 16, 8.0, 4.0
    xy = rng.uniform(0, 1, size=(5, 2)) * [lx, ly]
    spc = rng.integers(0, 2, size=5)
    ff = form_factor_table(["A", "B"])
    mask = pot.bandlimit_mask(nx, ny, lx, ly, 2.0 / 3.0)
    V0 = pot.slice_potential(xy, spc, ff, nx, ny, lx, ly, mask)
    p, q = 3, -2
    V1 = pot.slice_potential(xy + [p * lx / nx, q * ly / ny], spc, ff, nx, ny, lx, ly, mask)
    np.testing.assert_allclose(V1, np.roll(np.roll(V0, p, axis=1), q, axis=0), atol=1e-11)


def test_factorised_sum_equals_direct_loop():
    rng = np.random.default_rng(7)
    nx, ny, lx, ly = 16, 8, 4.0, 3.0
    xy = rng.uniform(-0.5, 1.5, size=(6, 2)) * [lx, ly]
    spc = rng.integers(0, 2, size=6)
    ff = form_factor_table(["A", "B"])
    for frac in (2.0 / 3.0, 0.0):
        mask = pot.bandlimit_mask(nx, ny, lx, ly, frac)
        a = pot.slice_potential_k(xy, spc, ff, nx, ny, lx, ly, mask)
        b = pot.slice_potential_k_direct(xy, spc, ff, nx, ny, lx, ly, mask)
        np.testing.assert_allclose(a, b, atol=1e-12 * np.max(np.abs(b)))


def test_bandlimit_mask_is_a_disc_of_the_smaller_nyquist():
    nx, ny, lx, ly = 64, 32, 16.0, 4.0        # k_N x = 2, k_N y = 4 -> min 2, kmax = 4/3
    m = pot.bandlimit_mask(nx, ny, lx, ly, 2.0 / 3.0)
    kx, ky = pot.k_vectors(nx, ny, lx, ly)
    assert m[0, 0] == 1
    # along x: |m|/16 < 4/3 -> |m| <= 21
    assert m[0, 21] == 1 and m[0, 22] == 0 and m[0, -21] == 1 and m[0, -22] == 0
    # along y: |n|/4 < 4/3 -> |n| <= 5
    assert m[5, 0] == 1 and m[6, 0] == 0
    # symmetric under k -> -k on the kept set (no Nyquist entries)
    assert m[:, nx // 2].sum() == 0 and m[ny // 2, :].sum() == 0


def test_potentials_bins_every_snapshot():
    spec = SimpleNamespace(nx=16, ny=16, lx=4.0, ly=4.0, dz=np.array([1.0, 1.0]), z0=0.0,
                           bandlimit=2.0 / 3.0)
    pos = np.array([[[1.0, 1.0, 0.5], [2.0, 2.0, 1.5], [3.0, 3.0, 2.5]],
                    [[1.0, 1.0, 1.5], [2.0, 2.0, 0.5], [3.0, 3.0, 1.0]]], dtype=np.float32)
    V, bins = pot.potentials(pos, np.array([0, 0, 0]), form_factor_table(["A"]), spec)
    np.testing.assert_array_equal(bins, [[0, 1, -1], [1, 0, 1]])
    # snapshot 1 slice 1 holds two atoms: its integral is twice that of one atom
    dxdy = (4.0 / 16) ** 2
    assert V[1, 1].sum() == pytest.approx(2 * V[1, 0].sum(), rel=1e-12)
    assert V[0, 0].sum() * dxdy == pytest.approx(
        TWO_PI_A0_E * pot.form_factor(FORM_FACTORS["A"], np.array([0.0]))[0], rel=1e-12)
