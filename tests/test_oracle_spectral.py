"""Pins of the oracle's dealiasing mask and spectral derivatives.

The mask is the cubic 2/3 rule (keep a mode iff 3|k_i| < n on every axis);
derivatives are exact for every retained Fourier mode.  Derivatives are
observed through the mass equation R_rho = -div(m), whose only ingredient is
the spectral derivative of a state field."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I


def retained(n):
    K = (n - 1) // 3
    return K


@pytest.mark.parametrize("n", [8, 12, 16, 24])
def test_mask_mode_count(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n, n))
    g = O.project(f)
    spec = np.fft.rfftn(g)
    K = retained(n)
    kept = np.abs(spec) > 1e-9 * np.abs(spec).max()
    assert kept.sum() == (K + 1) * (2 * K + 1) ** 2
    # every kept mode satisfies 3|k| < n on each axis
    kz, ky, kx = np.nonzero(kept)
    wz = np.where(2 * kz < n, kz, kz - n)
    wy = np.where(2 * ky < n, ky, ky - n)
    assert np.all(3 * np.abs(wz) < n) and np.all(3 * np.abs(wy) < n) and np.all(3 * kx < n)
    # projection is idempotent
    assert np.max(np.abs(O.project(g) - g)) < 1e-13 * np.abs(g).max()


@pytest.mark.parametrize("n,k", [(12, (3, 0, 0)), (12, (4, 0, 0)), (16, (5, -3, 2)), (16, (6, 0, 0)),
                                 (24, (7, 7, -7)), (24, (8, 1, 1)), (32, (10, 0, 3))])
def test_projection_single_mode(n, k):
    z, y, x = I.grid(n)
    f = np.cos(k[0] * x + k[1] * y + k[2] * z + 0.3) + 0 * x + 0 * y + 0 * z
    inband = all(3 * abs(c) < n for c in k)
    g = O.project(f)
    if inband:
        assert np.max(np.abs(g - f)) < 1e-13
    else:
        assert np.max(np.abs(g)) < 1e-13


@pytest.mark.parametrize("n", [12, 16, 24])
def test_derivative_of_every_inband_axis_mode(n):
    """m = e_j cos(k x_j + phi) gives R_rho = k sin(k x_j + phi) exactly for every
    retained k, and zero for the first dropped k."""
    K = retained(n)
    z, y, x = I.grid(n)
    coords = (x, y, z)
    for j in range(3):
        for k in list(range(1, K + 1)) + [K + 1]:
            U = np.zeros((8, n, n, n))
            U[0] = 1.0
            U[7] = 1.0
            U[1 + j] = np.cos(k * coords[j] + 0.4) + 0 * x + 0 * y + 0 * z
            R = O.rhs(U)
            expect = k * np.sin(k * coords[j] + 0.4) + 0 * x + 0 * y + 0 * z
            if k <= K:
                assert np.max(np.abs(R[0] - expect)) < 1e-12 * k
            else:
                assert np.max(np.abs(R[0])) < 1e-12


def test_derivative_oblique_mode():
    n = 16
    z, y, x = I.grid(n)
    kv = np.array([2, -3, 5])
    ph = kv[0] * x + kv[1] * y + kv[2] * z + 1.1
    U = np.zeros((8, n, n, n))
    U[0] = 1.0
    U[7] = 1.0
    a = np.array([0.3, -0.7, 0.2])
    for j in range(3):
        U[1 + j] = a[j] * np.cos(ph)
    R = O.rhs(U)
    expect = (a @ kv) * np.sin(ph)
    assert np.max(np.abs(R[0] - expect)) < 1e-12
