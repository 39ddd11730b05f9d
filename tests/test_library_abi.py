"""CPU checks of the C-ABI library: it loads, exports every function include/tacaw.h declares,
the Python binding covers the same names, host-side helpers agree with the oracle, and the CPU
emulation of the FFT plans matches a float64 DFT.  No kernel is launched."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tacaw.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tacaw_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2401_15599_amd as tw
    lib = ctypes.CDLL(tw.LIB_PATH)
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tw.EXPORTED)


def test_host_helpers_agree_with_oracle():
    import paper_2401_15599_amd as tw
    from oracle import physics
    for e in (60e3, 100e3, 200e3):
        assert tw.tacaw_wavelength(e) == pytest.approx(physics.wavelength(e), rel=1e-15)
        assert tw.tacaw_interaction_parameter(e) == pytest.approx(physics.interaction_parameter(e), rel=1e-15)
    np.testing.assert_allclose(tw.tacaw_energy_axis(256, 5.0), physics.energy_axis(256, 5.0), rtol=1e-14)


def test_errors_are_reported_without_a_device_call():
    import paper_2401_15599_amd as tw
    with pytest.raises(tw.TacawError):
        tw.tacaw_energy_axis(0, 5.0)


def test_fft_plans_cpu_emulation():
    exe = os.path.join(ROOT, "paper_2401_15599_amd", "fft_host_check")
    assert os.path.exists(exe), "run __graft_entry__.build() first"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    assert "FFT host check passed" in r.stdout
    # the odd-length plans (radices 4, 5, 7 and 10 with an in-place LDS last stage) are covered
    assert "n560" in r.stdout and "n1000" in r.stdout
    # the structure factor's fixed-point phase factors
    assert "phase_factor" in r.stdout


def test_plan_counts_cover_the_supported_grids():
    import paper_2401_15599_amd as tw
    for n in (16, 32, 64, 128, 256, 512, 1024, 560, 1000):
        assert tw.tacaw_plan_count(n) >= 1, n
    for n in (8, 48, 600, 2048):
        assert tw.tacaw_plan_count(n) == 0, n
