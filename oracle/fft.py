"""Library-free discrete Fourier transforms in FP64 (oracle).

Sign convention (the one implied by the paper's interpolation formulas, Eq.
pstd_psiinc and Eq. AnBottomPsi): forward F[x]_m = sum_j x_j exp(-2 pi i j m/N),
inverse (1/N) sum_m X_m exp(+2 pi i j m/N).

  naive_dft  the definition, O(N^2)
  fft        radix-2 recursion for N = 2^p, Bluestein's chirp-z (built on the
             radix-2 transform) for every other N, the naive sum for N <= 8.

A backend switch lets long physics runs take the FFT step from a library
(SciPy's pocketfft, same definition, optionally threaded over the batch of
pencils); the default is the library-free transform, which the tests pin to
the definition and to the library.

    with fft.backend("pocketfft", workers=16):
        ...   # every transform of the oracle inside goes through the library
"""
from __future__ import annotations

import contextlib

import numpy as np

BACKENDS = ("library-free", "pocketfft")
_backend = {"name": "library-free", "workers": 1}


def get_backend():
    """(name, workers) of the transform in use."""
    return _backend["name"], _backend["workers"]


def set_backend(name, workers=1):
    if name not in BACKENDS:
        raise ValueError(f"unknown FFT backend {name!r}")
    _backend["name"] = name
    _backend["workers"] = max(1, int(workers))


@contextlib.contextmanager
def backend(name, workers=1):
    """Use `name` for every transform inside the block, then restore."""
    old = get_backend()
    set_backend(name, workers)
    try:
        yield
    finally:
        set_backend(*old)


def naive_dft(x, axis=-1, inverse=False):
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    N = x.shape[-1]
    j = np.arange(N)
    sign = 1.0 if inverse else -1.0
    W = np.exp(sign * 2j * np.pi * (np.outer(j, j) % N) / N)
    y = x @ W  # y[..., m] = sum_j x[..., j] W[j, m]
    if inverse:
        y = y / N
    return np.moveaxis(y, -1, axis)


def _radix2(x, sign):
    N = x.shape[-1]
    if N == 1:
        return x.copy()
    even = _radix2(x[..., 0::2], sign)
    odd = _radix2(x[..., 1::2], sign)
    k = np.arange(N // 2)
    t = np.exp(sign * 2j * np.pi * k / N) * odd
    return np.concatenate([even + t, even - t], axis=-1)


def _bluestein(x, sign):
    # X_m = c_m sum_n (x_n c_n) conj(c_{m-n}),  c_n = exp(sign i pi n^2 / N)
    N = x.shape[-1]
    M = 1
    while M < 2 * N - 1:
        M *= 2
    n = np.arange(N)
    c = np.exp(sign * 1j * np.pi * ((n * n) % (2 * N)) / N)
    a = np.zeros(x.shape[:-1] + (M,), dtype=np.complex128)
    a[..., :N] = x * c
    b = np.zeros(M, dtype=np.complex128)
    b[:N] = np.conj(c)
    b[M - N + 1:] = np.conj(c[1:][::-1])
    A = _radix2(a, -1.0)
    B = _radix2(b, -1.0)
    conv = _radix2(A * B, 1.0) / M
    return c * conv[..., :N]


def _lastaxis(x, sign):
    N = x.shape[-1]
    if _backend["name"] == "pocketfft":
        import scipy.fft as sfft
        w = _backend["workers"]
        return sfft.fft(x, axis=-1, workers=w) if sign < 0 else sfft.ifft(x, axis=-1, workers=w) * N
    if N <= 8:
        W = np.exp(sign * 2j * np.pi * (np.outer(np.arange(N), np.arange(N)) % N) / N)
        return x @ W
    if N & (N - 1) == 0:
        return _radix2(x, sign)
    return _bluestein(x, sign)


def fft(x, axis=-1):
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_lastaxis(x, -1.0), -1, axis)


def ifft(X, axis=-1):
    X = np.moveaxis(np.asarray(X, dtype=np.complex128), axis, -1)
    N = X.shape[-1]
    return np.moveaxis(_lastaxis(X, 1.0) / N, -1, axis)


def fft2(x, axes=(-2, -1)):
    return fft(fft(x, axes[0]), axes[1])
