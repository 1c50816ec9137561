"""Pins of the kinematic-dynamo theory in tests/dynamo_theory.py, which the
GPU dynamo runs are held to, and through it of the oracle's kinematic mode.

* With no flow the matrix is the diagonal of the resistive decay rates
  -eta |k|^2 (closed form).
* The 1:1:1 ABC flow has a first dynamo window: fields grow for
  8.9 < Rm < 17.5 (Rm = U0 / (eta k_f)); the onset at 8.9 is Arnold and
  Korkina's (1983), the end at 17.5 Galloway and Frisch's (1986).  The
  leading growth rate must change sign across both, and its value at onset
  must not move between two truncations (converged).
* The matrix applied to a field equals the oracle's kinematic right-hand
  side of B for a flow with three different amplitudes A, B, C, mode by
  mode (so a swapped component or a sign would show), and the oracle leaves
  rho, m and E unchanged in that mode.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I
from tests import dynamo_theory as D


def test_no_flow_gives_the_diffusion_rates():
    n, eta = 9, 0.37
    M = D.induction_matrix(n, eta, 0.0, 0.0, 0.0).toarray()
    ks, K = D.band_modes(n)
    assert K == 2 and len(ks) == 5 ** 3 - 1
    want = -eta * np.repeat(np.sum(ks.astype(float) ** 2, axis=1), 2)
    assert np.array_equal(M, np.diag(want))


def test_first_dynamo_window_of_the_111_flow():
    # onset at Rm = 8.9: converged already at n = 24 (|k_i| <= 7)
    below = D.leading_eigenvalues(24, 1.0 / 8.8, 2, tol=1e-8)[0]
    above = D.leading_eigenvalues(24, 1.0 / 9.0, 2, tol=1e-8)[0]
    above32 = D.leading_eigenvalues(32, 1.0 / 9.0, 2, tol=1e-8)[0]
    assert below.real < -5e-4 and above.real > 2e-4
    assert abs(above32.real - above.real) < 1e-6 and abs(abs(above32.imag) - abs(above.imag)) < 1e-6
    # end at Rm = 17.5 (n = 32, |k_i| <= 10)
    inside = D.leading_eigenvalues(32, 1.0 / 17.3, 2, tol=1e-8)[0]
    outside = D.leading_eigenvalues(32, 1.0 / 17.7, 2, tol=1e-8)[0]
    assert inside.real > 1e-4 and outside.real < -1e-4


def _band_coefficients(f, n):
    """Fourier coefficients (1/n^3) sum f e^{-ik.x} of a field (3, n, n, n)
    indexed [z][y][x] at the band modes, as (modes, 3)."""
    ks, _ = D.band_modes(n)
    out = np.empty((len(ks), 3), complex)
    for c in range(3):
        F = np.fft.fftn(f[c]) / n ** 3
        out[:, c] = F[ks[:, 2] % n, ks[:, 1] % n, ks[:, 0] % n]
    return ks, out


@pytest.mark.parametrize("abc", [(1.0, 0.7, 0.4), (0.3, 1.0, 0.6)])
def test_matrix_is_the_oracle_kinematic_rhs(abc):
    n, eta, gamma = 12, 0.05, 5.0 / 3.0
    A, B, C = abc
    u = I.abc_flow(n, A, B, C)
    Bf = I.random_field(n, 7, 3, 1, 3, 0.3)
    rho = np.ones((n, n, n))
    U = I.conserved(rho, u, Bf, np.full((n, n, n), 2.0), gamma)
    R = O.rhs(U, gamma, 0.01, eta, options=O.KINEMATIC)
    assert np.all(R[:4] == 0) and np.all(R[7] == 0)
    ks, bh = _band_coefficients(Bf, n)
    _, rh = _band_coefficients(R[4:7], n)
    E = np.stack([D._basis(k) for k in ks])  # (m, 2, 3)
    # the field is solenoidal, so its two transverse components carry it whole
    assert np.max(np.abs(np.einsum("mc,mc->m", bh, ks.astype(float)))) < 1e-12
    b = np.einsum("msc,mc->ms", E, bh).reshape(-1)
    got = np.einsum("msc,mc->ms", E, rh).reshape(-1)
    want = D.induction_matrix(n, eta, A, B, C) @ b
    assert np.max(np.abs(want)) > 0.05
    assert np.max(np.abs(got - want)) < 1e-14
    # and the oracle's right-hand side has no component along k
    assert np.max(np.abs(np.einsum("mc,mc->m", rh, ks.astype(float)))) < 1e-12
