"""Dense discrete Fourier transforms (oracle, complex128).

F[a, b] = exp(-2 pi i a b / N) is the unnormalised forward DFT; the inverse is conj(F) / N.
No fast algorithm is used anywhere in the oracle: every transform is a matrix product, so it can be
checked against the definition by eye (and against a library FFT in the tests).
"""
import numpy as np


def dft_matrix(n):
    """Forward DFT matrix exp(-2 pi i a b / n), complex128 [n][n].

    The exponent a*b is reduced modulo n in integers first, so the phase argument stays exact."""
    a = np.arange(n)
    ab = np.outer(a, a) % n
    return np.exp(-2j * np.pi * ab / n)


def fftfreq_index(n):
    """Signed frequency index m of each DFT bin in storage order: 0..n/2-1, -n/2..-1."""
    m = np.arange(n)
    return np.where(m < (n + 1) // 2, m, m - n)


def dft2(x):
    """Unnormalised 2-D forward DFT over the last two axes ([..., y, x])."""
    fy = dft_matrix(x.shape[-2])
    fx = dft_matrix(x.shape[-1])
    return fy @ x @ fx


def idft2(x):
    """Unnormalised 2-D inverse DFT (exp(+2 pi i ...), no 1/N) over the last two axes."""
    fy = dft_matrix(x.shape[-2]).conj()
    fx = dft_matrix(x.shape[-1]).conj()
    return fy @ x @ fx


def dft_axis(x, axis, inverse=False):
    """Unnormalised 1-D DFT along one axis (forward exp(-2 pi i k t / n) unless inverse)."""
    n = x.shape[axis]
    f = dft_matrix(n)
    if inverse:
        f = f.conj()
    xm = np.moveaxis(x, axis, -1)
    return np.moveaxis(xm @ f, -1, axis)
