"""Pins of the oracle's library-free FFTs against the DFT definition, an
independent library (numpy's pocketfft), Parseval and the round trip; and of
the library backend (SciPy's pocketfft, threaded) that long runs may select,
against the library-free transform and the definition."""
import numpy as np
import pytest

from oracle import fft

LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16, 17, 24, 32, 48, 64, 96, 100, 128, 160]


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 11, 16, 20])
def test_naive_dft_matches_numpy(N):
    rng = np.random.default_rng(N)
    x = rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N))
    assert np.allclose(fft.naive_dft(x), np.fft.fft(x), rtol=0, atol=1e-12 * max(1, N))
    assert np.allclose(fft.naive_dft(x, inverse=True), np.fft.ifft(x), rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", LENGTHS)
def test_fft_matches_definition(N):
    rng = np.random.default_rng(100 + N)
    x = rng.normal(size=(3, N)) + 1j * rng.normal(size=(3, N))
    ref = fft.naive_dft(x)
    got = fft.fft(x)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max() * max(1, np.log2(max(N, 2)))
    assert np.abs(fft.ifft(got) - x).max() <= 1e-13 * np.abs(x).max() * max(1, np.log2(max(N, 2)))


@pytest.mark.parametrize("N", [48, 160, 288])
def test_fft_matches_library_and_parseval(N):
    rng = np.random.default_rng(7)
    x = rng.normal(size=(2, N)) + 1j * rng.normal(size=(2, N))
    X = fft.fft(x)
    assert np.abs(X - np.fft.fft(x)).max() <= 1e-12 * np.abs(X).max()
    assert abs(np.sum(np.abs(X) ** 2) / N - np.sum(np.abs(x) ** 2)) <= 1e-12 * np.sum(np.abs(x) ** 2)


def test_fft_along_axis():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(6, 10, 12)) + 1j * rng.normal(size=(6, 10, 12))
    for ax in range(3):
        assert np.allclose(fft.fft(x, axis=ax), np.fft.fft(x, axis=ax), atol=1e-12)
        assert np.allclose(fft.ifft(x, axis=ax), np.fft.ifft(x, axis=ax), atol=1e-13)


@pytest.mark.parametrize("N", [12, 48, 160, 288])
@pytest.mark.parametrize("workers", [1, 4])
def test_library_backend_matches_library_free(N, workers):
    rng = np.random.default_rng(N + workers)
    x = rng.normal(size=(5, 3, N)) + 1j * rng.normal(size=(5, 3, N))
    ref_f, ref_i = fft.fft(x, axis=2), fft.ifft(x, axis=0)
    assert fft.get_backend() == ("library-free", 1)
    with fft.backend("pocketfft", workers=workers):
        assert fft.get_backend() == ("pocketfft", workers)
        got_f, got_i = fft.fft(x, axis=2), fft.ifft(x, axis=0)
    assert fft.get_backend() == ("library-free", 1)
    assert np.abs(got_f - ref_f).max() <= 1e-12 * np.abs(ref_f).max()
    assert np.abs(got_i - ref_i).max() <= 1e-12 * np.abs(ref_i).max()
    # and against the definition directly
    assert np.abs(got_f - fft.naive_dft(x, axis=2)).max() <= 1e-12 * np.abs(ref_f).max()


def test_unknown_backend_is_refused():
    with pytest.raises(ValueError):
        fft.set_backend("fftw")
