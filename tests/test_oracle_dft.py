"""The oracle's dense DFT matrices against numpy's FFT (an independent library routine)."""
import numpy as np

from oracle import dft


def test_dense_dft_matches_numpy_fft():
    rng = np.random.default_rng(0)
    for n in (1, 2, 8, 16, 30, 64):
        x = rng.normal(size=(3, n)) + 1j * rng.normal(size=(3, n))
        np.testing.assert_allclose(x @ dft.dft_matrix(n), np.fft.fft(x, axis=-1), atol=1e-12 * n)
        np.testing.assert_allclose(dft.dft_axis(x, 1, inverse=True), np.fft.ifft(x, axis=-1) * n,
                                   atol=1e-12 * n)


def test_dense_dft2_matches_numpy_fft2():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 16, 32)) + 1j * rng.normal(size=(2, 16, 32))
    np.testing.assert_allclose(dft.dft2(x), np.fft.fft2(x), atol=1e-11)
    np.testing.assert_allclose(dft.idft2(x), np.fft.ifft2(x) * 512, atol=1e-11)


def test_fftfreq_index():
    for n in (8, 9, 64):
        np.testing.assert_array_equal(dft.fftfreq_index(n), np.round(np.fft.fftfreq(n) * n))
