"""Pins of the oracle's scalar physics: the paper's printed energy-axis numbers, textbook electron
wavelengths, and the detailed-balance property of the Kubo factor."""
import math
import os

import numpy as np
import pytest

from oracle import physics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "energy_axis.txt")


def _rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append(dict(name=f[0], dt=float(f[1]), T=int(f[2]), n_e=int(f[3]), hop=int(f[4]),
                         segs=int(f[5]), thz=float(f[6]), mev=float(f[7]), ps=float(f[8])))
    return rows


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r["name"])
def test_energy_axis_matches_printed_numbers(row):
    # Nyquist frequency 1/(2 dt) and energy pi hbar/dt, as printed (rounded) in the footnotes
    assert physics.nyquist_thz(row["dt"]) == pytest.approx(row["thz"], rel=1e-3)
    assert physics.e_max(row["dt"]) * 1e3 == pytest.approx(row["mev"], abs=0.5)
    # segment duration n_e * dt
    assert row["n_e"] * row["dt"] / 1000.0 == pytest.approx(row["ps"], rel=1e-9)
    if row["segs"] > 0:
        assert physics.n_segments(row["T"], row["n_e"], row["hop"]) == row["segs"]
    # the ascending axis ends one bin below +E_max and starts at -E_max (even n_e)
    ax = physics.energy_axis(row["n_e"], row["dt"])
    if row["n_e"] % 2 == 0:
        assert ax[0] == pytest.approx(-physics.e_max(row["dt"]), rel=1e-12)
    assert ax[row["n_e"] // 2] == 0.0
    assert ax[1] - ax[0] == pytest.approx(physics.e_min(row["n_e"], row["dt"]), rel=1e-12)


def test_si_snapshots_used_twice_except_ends():
    # Si footnote: with 79 sets of 100 offset by 50, all 4000 snapshots are used twice except the
    # first and the last 50.
    T, n_e, hop = 4000, 100, 50
    use = np.zeros(T, int)
    for g in range(physics.n_segments(T, n_e, hop)):
        use[g * hop: g * hop + n_e] += 1
    assert np.all(use[:50] == 1) and np.all(use[-50:] == 1) and np.all(use[50:-50] == 2)


def test_wavelengths_textbook_values():
    # relativistic electron wavelengths tabulated in electron-microscopy textbooks
    assert physics.wavelength(100e3) == pytest.approx(0.037014, abs=2e-6)
    assert physics.wavelength(200e3) == pytest.approx(0.025079, abs=2e-6)
    assert physics.wavelength(300e3) == pytest.approx(0.019687, abs=2e-6)
    # non-relativistic limit lambda -> h / sqrt(2 m E) at low energy
    e = 10.0
    nonrel = physics.HC_EV_A / math.sqrt(2.0 * physics.M0C2_EV * e)
    assert physics.wavelength(e) == pytest.approx(nonrel, rel=1e-5)


def test_interaction_parameter_limits():
    # sigma = 2 pi m e lambda / h^2 with relativistic mass: sigma lambda E -> 2 pi (m0c^2+E)/(2m0c^2+E)
    # tends to pi at low energy and to 2 pi at very high energy
    for e, lim in ((1.0, math.pi), (1e12, 2.0 * math.pi)):
        s = physics.interaction_parameter(e)
        assert s * physics.wavelength(e) * e == pytest.approx(lim, rel=1e-5)
    assert physics.interaction_parameter(100e3) == pytest.approx(9.244e-4, rel=1e-3)


def test_kubo_detailed_balance_and_limits():
    T = 300.0
    beta = 1.0 / (physics.KB_EV_K * T)
    e = np.linspace(-0.4, 0.4, 801)
    k = physics.kubo_factor(e, T)
    kneg = physics.kubo_factor(-e, T)
    np.testing.assert_allclose(k / kneg, np.exp(beta * e), rtol=1e-12)
    assert physics.kubo_factor(np.array([0.0]), T)[0] == 1.0
    # continuity across the series / closed-form switch
    # both sides of the series / closed-form switch agree with the Taylor series of x/(1-e^-x)
    y = np.array([0.5e-4, 0.99e-4, 1.01e-4, 2e-4, -1.01e-4])
    kk = physics.kubo_factor(y / beta, T)
    np.testing.assert_allclose(kk, 1 + y / 2 + y ** 2 / 12 - y ** 4 / 720, rtol=1e-14)
    # classical (high temperature) limit -> 1; large loss -> beta E
    assert physics.kubo_factor(np.array([1e-3]), 1e9)[0] == pytest.approx(1.0, abs=1e-7)
    assert physics.kubo_factor(np.array([1.0]), T)[0] == pytest.approx(beta, rel=1e-12)
