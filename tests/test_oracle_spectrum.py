"""Pins of the oracle's time auto-correlation spectrum: brute-force correlation, library FFT,
Parseval/sum rule, static-lattice delta, loss/gain sign, normalisation and an exact closed form
for a rigidly shifted crystal."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import spectrum as sp
from oracle import multislice as ms
from oracle import potential as pot
from oracle.physics import energy_axis, kubo_factor, n_segments, HBAR_EV_FS
from workloads import fcc_cubic, rigid_shift_trajectory, form_factor_table


def _rand_stack(T, P, ny, nx, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(T, P, ny, nx)) + 1j * rng.normal(size=(T, P, ny, nx))


def test_periodogram_equals_bruteforce_autocorrelation():
    x = _rand_stack(11, 2, 3, 4, 0)
    for n_e, hop in ((8, 3), (4, 4), (11, 1)):
        np.testing.assert_allclose(sp.segment_periodogram(x, n_e, hop),
                                   sp.segment_periodogram_bruteforce(x, n_e, hop), rtol=1e-11)


def test_periodogram_matches_library_fft():
    x = _rand_stack(16, 1, 2, 2, 1)
    ref = np.abs(np.fft.fft(x[:8], axis=0)) ** 2 + np.abs(np.fft.fft(x[8:], axis=0)) ** 2
    np.testing.assert_allclose(sp.segment_periodogram(x, 8, 8), ref[:, 0] / 2, rtol=1e-12)


def test_parseval_sum_rule():
    # sum over energies of segment g = n_e * sum_{t in g} |phi(q,t)|^2: the energy-integrated
    # Kubo-transformed spectrum is the QEP mean intensity over the same snapshots
    x = _rand_stack(20, 3, 4, 4, 2)
    n_e, hop = 8, 5
    G = n_segments(20, n_e, hop)
    P = sp.segment_periodogram(x, n_e, hop)
    qep = sum(np.sum(np.abs(x[g * hop:g * hop + n_e]) ** 2, axis=(0, 1)) for g in range(G)) / G
    np.testing.assert_allclose(P.sum(axis=0), n_e * qep, rtol=1e-12)


def test_static_lattice_gives_a_delta_at_zero_energy():
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(1, 2, 4, 4)) + 1j * rng.normal(size=(1, 2, 4, 4))
    x = np.repeat(phi, 16, axis=0)
    S, Z = sp.spectrum(x, 16, 16, 5.0, 300.0)
    assert np.max(np.abs(np.delete(S, 8, axis=0))) < 1e-15
    full = np.fft.fftshift(np.sum(np.abs(phi[0]) ** 2, axis=0))
    np.testing.assert_allclose(S[8], full / full.sum(), rtol=1e-12)


def test_loss_side_is_positive_energy():
    # phi(t) = exp(+i E0 t/hbar): the spectral sum puts this at E = +E0 (a loss) because the
    # energy kernel is exp(-i E t/hbar) and phi(t) carries exp(+i (E_m - E_n) t/hbar)
    n_e, dt, k0 = 32, 5.0, 5
    e0 = 2 * math.pi * HBAR_EV_FS * k0 / (n_e * dt)
    t = np.arange(n_e) * dt
    x = np.exp(1j * e0 * t / HBAR_EV_FS)[:, None, None, None] * np.ones((1, 1, 2, 2))
    S, _ = sp.spectrum(x, n_e, n_e, dt, 300.0)
    e = energy_axis(n_e, dt)
    j = np.argmax(S[:, 0, 0])
    assert e[j] == pytest.approx(e0, rel=1e-12) and e[j] > 0
    assert np.sum(S[j]) == pytest.approx(1.0, rel=1e-12)


def test_normalisation_crop_and_kubo_ratio():
    x = _rand_stack(24, 2, 8, 6, 4)
    n_e, hop, dt, T = 8, 8, 7.5, 300.0
    S, Z = sp.spectrum(x, n_e, hop, dt, T)
    assert S.sum() == pytest.approx(1.0, rel=1e-12)
    Sc, Zc = sp.spectrum(x, n_e, hop, dt, T, nqy=3, nqx=4)
    assert Zc == Z
    np.testing.assert_array_equal(Sc, S[:, 4 - 1:4 + 2, 3 - 2:3 + 2])
    ct = sp.kubo_transformed_spectrum(x, n_e, hop)
    ratio = S * Z / ct
    np.testing.assert_allclose(ratio, kubo_factor(energy_axis(n_e, dt), T)[:, None, None]
                               * np.ones_like(ratio), rtol=1e-12)


def test_rigid_shift_spectrum_closed_form():
    # a crystal shifted rigidly by p(t) pixels: S(q, E) = |phi_0(q)|^2 |DFT_t exp(-2 pi i q_x p(t) dx)|^2
    st = fcc_cubic(4.0, (2, 2, 2))
    nx = ny = 32
    lx = st.cell[0]
    spec = SimpleNamespace(nx=nx, ny=ny, lx=lx, ly=st.cell[1], dz=np.array([4.0, 4.0]), z0=0.0,
                           bandlimit=2.0 / 3.0)
    T, n_e = 16, 16
    pos, p = rigid_shift_trajectory(st, T, lx / nx, seed=9)
    V, _ = pot.potentials(pos, st.species, form_factor_table(["A"]), spec)
    beam = SimpleNamespace(probe=False, energy_ev=100e3)
    ex = ms.exit_waves(V, spec, beam)
    P = sp.segment_periodogram(ex, n_e, n_e)
    static = pos[:1] - np.array([p[0] * lx / nx, 0, 0], dtype=np.float32)
    phi0 = ms.exit_waves(pot.potentials(static, st.species, form_factor_table(["A"]), spec)[0],
                         spec, beam)[0, 0]
    qx = np.fft.fftfreq(nx, d=lx / nx)
    phase = np.exp(-2j * math.pi * qx[None, :] * (p[:, None] * lx / nx))      # [T][nx]
    per_qx = np.abs(np.fft.fft(phase, axis=0)) ** 2                            # [n_e][nx]
    ref = np.abs(phi0)[None] ** 2 * per_qx[:, None, :]
    np.testing.assert_allclose(P, ref, atol=1e-11 * ref.max())
