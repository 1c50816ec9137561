"""Pins of the oracle FFT against the DFT's definition (brute force), against
numpy.fft (pocketfft, run as a library) and against Parseval / inversion."""
import numpy as np
import pytest

from oracle import oracle as O


def brute_dft(x, sign=-1):
    n = len(x)
    j = np.arange(n)
    W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return W @ x


def smooth_lengths():
    out = []
    for a in range(0, 7):
        for b in range(0, 5):
            n = 2 ** a * 3 ** b
            if 1 <= n <= 96:
                out.append(n)
    return sorted(out)


@pytest.mark.parametrize("n", smooth_lengths() + [5, 7, 11, 13, 97])
def test_fft1d_matches_brute_force(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    scale = np.linalg.norm(x) * np.sqrt(n)
    for sign in (-1, 1):
        got = O.fft1d(x, sign)
        ref = brute_dft(x, sign)
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale


def test_plane_wave_and_delta():
    n = 48
    k = 7
    x = np.exp(2j * np.pi * k * np.arange(n) / n)
    X = O.fft1d(x, -1)
    expect = np.zeros(n, complex)
    expect[k] = n
    assert np.max(np.abs(X - expect)) < 1e-12
    d = np.zeros(n, complex)
    d[0] = 1.0
    assert np.max(np.abs(O.fft1d(d, -1) - 1.0)) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_fft3d_matches_brute_force(n):
    rng = np.random.default_rng(100 + n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    idx = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / n)
    # explicit triple sum over (z, y, x) for every (kz, ky, kx)
    ref = np.einsum("az,by,cx,zyx->abc", W, W, W, a)
    got = O.fft3d(a, -1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n", [16, 24, 32, 48])
def test_fft3d_matches_numpy(n):
    rng = np.random.default_rng(7 * n)
    a = rng.standard_normal((n, n, n))
    got = O.fft3d(a, -1)
    ref = np.fft.fftn(a)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.abs(ref).max()
    back = O.fft3d(got, 1) / n ** 3
    assert np.max(np.abs(back - a)) <= 1e-13 * np.abs(a).max()


def test_parseval_3d():
    n = 24
    rng = np.random.default_rng(3)
    a = rng.standard_normal((n, n, n))
    A = O.fft3d(a, -1)
    lhs = np.sum(a * a)
    rhs = np.sum(np.abs(A) ** 2) / n ** 3
    assert abs(lhs - rhs) <= 1e-13 * lhs


def test_rejects_bad_arguments():
    with pytest.raises(RuntimeError):
        O.fft1d(np.zeros(0, complex), -1)
    with pytest.raises(RuntimeError):
        O.fft1d(np.zeros(4, complex), 0)
