"""Pins of the oracle's multislice: Fresnel closed form, unitarity, weak-phase limit, exact
lateral-shift equivariance of the full dynamical propagation, and the probe's position."""
import math
from types import SimpleNamespace

import numpy as np

from oracle import multislice as ms
from oracle import potential as pot
from oracle.dft import dft2, idft2
from oracle.physics import wavelength, interaction_parameter
from workloads import form_factor_table, fcc_cubic, rigid_shift_trajectory


def _spec(nx, ny, lx, ly, dz, bandlimit=2.0 / 3.0):
    return SimpleNamespace(nx=nx, ny=ny, lx=lx, ly=ly, dz=np.asarray(dz, float), z0=0.0,
                           bandlimit=bandlimit)


def _real_space_exit(phi, spec):
    n = spec.nx * spec.ny
    return idft2(phi * math.sqrt(n)) / n


def test_fresnel_gaussian_closed_form():
    # free-space propagation of exp(-r^2/2s^2) over z: s^2/s'^2 exp(-r^2/2s'^2), s'^2 = s^2 + i lam z/2pi.
    # A flipped propagator sign gives the complex conjugate width and fails by O(1).
    e, s, z = 100e3, 2.0, 1000.0
    spec = _spec(256, 256, 64.0, 64.0, [z], bandlimit=0.0)
    lam = wavelength(e)
    x = np.arange(256) * 0.25
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = (X - 32.0) ** 2 + (Y - 32.0) ** 2
    psi0 = np.exp(-r2 / (2 * s * s)).astype(np.complex128)
    phi = ms.propagate(psi0, np.zeros((1, 256, 256)), spec, e)
    got = _real_space_exit(phi, spec)
    s2 = s * s + 1j * lam * z / (2 * math.pi)
    ref = (s * s / s2) * np.exp(-r2 / (2 * s2))
    assert np.max(np.abs(got - ref)) < 1e-10
    wrong = (s * s / np.conj(s2)) * np.exp(-r2 / (2 * np.conj(s2)))
    assert np.max(np.abs(got - wrong)) > 0.1


def test_unitarity_without_band_limit_and_loss_with_it():
    rng = np.random.default_rng(11)
    spec = _spec(32, 32, 8.0, 8.0, np.full(100, 1.5), bandlimit=0.0)
    V = rng.uniform(0, 40.0, size=(100, 32, 32))
    phi = ms.propagate(ms.plane_wave(spec), V, spec, 100e3)
    assert abs(np.sum(np.abs(phi) ** 2) - 1.0) < 1e-12
    spec.bandlimit = 2.0 / 3.0
    _, states = ms.propagate(ms.plane_wave(spec), V, spec, 100e3, keep_states=True)
    norms = np.sum(np.abs(states) ** 2, axis=(1, 2))
    assert np.all(np.diff(norms) <= 1e-13) and norms[-1] < norms[0]


def test_weak_phase_single_slice_limit():
    # one slice of zero thickness: phi(k)/(i eps sigma) -> M(k) V(k) for k != 0, error O(eps)
    rng = np.random.default_rng(12)
    nx, ny, lx, ly = 32, 32, 8.0, 8.0
    spec = _spec(nx, ny, lx, ly, [0.0])
    ff = form_factor_table(["A", "B"])
    xy = rng.uniform(0, 1, size=(6, 2)) * [lx, ly]
    spc = rng.integers(0, 2, size=6)
    mask = pot.bandlimit_mask(nx, ny, lx, ly, spec.bandlimit)
    vk = pot.slice_potential_k(xy, spc, ff, nx, ny, lx, ly, mask)
    V = idft2(vk).real
    sigma = interaction_parameter(100e3)
    errs = []
    for eps in (1e-3, 1e-4):
        phi = ms.propagate(ms.plane_wave(spec), eps * V[None], spec, 100e3)
        est = phi / (1j * eps * sigma)
        est[0, 0] = 0.0
        ref = vk.copy()
        ref[0, 0] = 0.0
        errs.append(np.linalg.norm(est - ref) / np.linalg.norm(ref))
        # k = 0: 1 + i eps sigma V(0) + O(eps^2)
        assert abs(phi[0, 0] - (1 + 1j * eps * sigma * vk[0, 0])) < 10 * (eps * sigma * abs(vk[0, 0])) ** 2
    assert errs[0] < 0.05
    assert 5.0 < errs[0] / errs[1] < 20.0


def test_rigid_integer_pixel_shift_equivariance():
    # all atoms shifted by p(t) pixels along x under plane-wave illumination:
    # phi(q, t) = phi_0(q) exp(-2 pi i q_x p(t) dx), exactly (full dynamical multislice)
    st = fcc_cubic(4.0, (2, 2, 2))
    nx = ny = 32
    lx, ly = st.cell[0], st.cell[1]
    spec = _spec(nx, ny, lx, ly, [4.0, 4.0])
    pos, p = rigid_shift_trajectory(st, 4, lx / nx, seed=3)
    V, bins = pot.potentials(pos, st.species, form_factor_table(["A"]), spec)
    beam = SimpleNamespace(probe=False, energy_ev=100e3)
    ex = ms.exit_waves(V, spec, beam)[:, 0]
    _, base = rigid_shift_trajectory(st, 1, lx / nx, seed=3)
    phi0 = ms.exit_waves(pot.potentials(pos[:1] - [p[0] * lx / nx, 0, 0], st.species,
                                        form_factor_table(["A"]), spec)[0], spec, beam)[0, 0]
    qx = np.fft.fftfreq(nx, d=lx / nx)
    for t in range(4):
        ref = phi0 * np.exp(-2j * math.pi * qx[None, :] * p[t] * lx / nx)
        np.testing.assert_allclose(ex[t], ref, atol=1e-12)
    assert np.abs(ex[0]).max() > 0.05


def test_probe_is_normalised_and_centred_on_its_position():
    spec = _spec(128, 128, 32.0, 32.0, [2.0])
    beam = SimpleNamespace(probe=True, energy_ev=100e3, alpha_rad=0.03, defocus_a=0.0, cs_a=0.0,
                           probe_xy=np.array([[13.0, 17.5]]))
    psi = ms.initial_waves(spec, beam)[0]
    assert abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-12
    x = np.arange(128) * 0.25
    X, Y = np.meshgrid(x, x, indexing="xy")
    w = np.abs(psi) ** 2
    assert abs(np.sum(w * X) - 13.0) < 0.05 and abs(np.sum(w * Y) - 17.5) < 0.05
    # the intensity peak sits on the pixel of the position
    iy, ix = np.unravel_index(np.argmax(w), w.shape)
    assert (ix, iy) == (52, 70)
    # spectrum confined to the aperture lambda |k| <= alpha
    a = dft2(psi)
    kx = np.fft.fftfreq(128, d=0.25)
    k = np.hypot(kx[None, :], kx[:, None])
    assert np.max(np.abs(a[k * wavelength(100e3) > 0.0301])) < 1e-10


def test_probe_defocus_equals_free_space_propagation_of_the_focused_probe():
    # chi's defocus term pi lambda df k^2 is exactly the phase of the (already pinned) Fresnel
    # propagator over a thickness df: the probe at defocus df is the in-focus probe propagated
    # forward by df in vacuum.  A wrong sign or factor of the defocus term fails by O(1).
    spec = _spec(128, 128, 32.0, 32.0, [1.0], bandlimit=0.0)
    pos = np.array([[13.0, 17.5]])
    for e, alpha, df in ((100e3, 0.03, 50.0), (200e3, 0.02, -120.0)):
        focused = SimpleNamespace(probe=True, energy_ev=e, alpha_rad=alpha, defocus_a=0.0,
                                  cs_a=0.0, probe_xy=pos)
        defocused = SimpleNamespace(probe=True, energy_ev=e, alpha_rad=alpha, defocus_a=df,
                                    cs_a=0.0, probe_xy=pos)
        psi_f = ms.initial_waves(spec, focused)[0]
        psi_d = ms.initial_waves(spec, defocused)[0]
        n = spec.nx * spec.ny
        spec.dz = np.array([df])
        phi = ms.propagate(psi_f, np.zeros((1, 128, 128)), spec, e)
        np.testing.assert_allclose(phi, dft2(psi_d) / math.sqrt(n), atol=1e-12)
        spec.dz = np.array([-df])
        wrong = ms.propagate(psi_f, np.zeros((1, 128, 128)), spec, e)
        assert np.max(np.abs(wrong - dft2(psi_d) / math.sqrt(n))) > 1e-2


def _probe_spectrum_at_origin(spec, e, alpha, df, cs):
    beam = SimpleNamespace(probe=True, energy_ev=e, alpha_rad=alpha, defocus_a=df, cs_a=cs,
                           probe_xy=np.array([[0.0, 0.0]]))
    a = dft2(ms.initial_waves(spec, beam)[0])
    kx = np.fft.fftfreq(spec.nx, d=spec.lx / spec.nx)
    ky = np.fft.fftfreq(spec.ny, d=spec.ly / spec.ny)
    return a, kx, ky


def test_probe_aberration_phase_matches_the_angle_form():
    # textbook aberration function in terms of the scattering angle theta = lambda |k|:
    # chi(theta) = (2 pi / lambda) (Cs theta^4 / 4 + df theta^2 / 2); the probe's spectrum at the
    # origin is A(k) exp(-i chi) times a positive constant.  Checked with Cs = 1.2 mm and 0.5 mm.
    spec = _spec(128, 128, 48.0, 48.0, [1.0], bandlimit=0.0)
    for e, alpha, df, cs in ((100e3, 0.025, -50.0, 1.2e7), (200e3, 0.02, 35.0, 5.0e6)):
        lam = wavelength(e)
        a, kx, ky = _probe_spectrum_at_origin(spec, e, alpha, df, cs)
        assert a[0, 0].real > 0 and abs(a[0, 0].imag) < 1e-12 * a[0, 0].real
        theta = lam * np.hypot(kx[None, :], ky[:, None])
        inside = theta <= alpha
        chi = (2 * math.pi / lam) * (cs * theta ** 4 / 4 + df * theta ** 2 / 2)
        ratio = a / a[0, 0]
        assert np.max(np.abs(ratio[inside] - np.exp(-1j * chi[inside]))) < 1e-9
        assert np.max(np.abs(a[~inside])) < 1e-12
        assert np.max(chi[inside]) > 20.0          # the Cs term is far from negligible here


def test_spherical_aberration_shifts_the_focus_of_a_ring_by_cs_theta_squared():
    # longitudinal spherical aberration: the part of the probe at angle theta behaves like a
    # defocus df + Cs theta^2.  For two k points on neighbouring rings the phase difference
    # divided by pi lambda (k2^2 - k1^2) is exactly df + Cs (theta1^2 + theta2^2) / 2 (the secant
    # of a quadratic in k^2); phases are compared as small differences, so no unwrapping.
    spec = _spec(128, 128, 48.0, 48.0, [1.0], bandlimit=0.0)
    e, alpha, df, cs = 100e3, 0.025, -50.0, 1.2e7
    lam = wavelength(e)
    a, kx, ky = _probe_spectrum_at_origin(spec, e, alpha, df, cs)
    checked = 0
    for m in range(1, 20):
        k1, k2 = kx[m] ** 2, kx[m] ** 2 + ky[1] ** 2
        if lam * math.sqrt(k2) > alpha:
            break
        dphase = -np.angle(a[1, m] / a[0, m])
        slope = dphase / (math.pi * lam * (k2 - k1))
        assert abs(slope - (df + cs * lam ** 2 * (k1 + k2) / 2)) < 1e-6 * abs(cs * lam ** 2 * k2)
        checked += 1
    assert checked >= 10
