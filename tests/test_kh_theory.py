"""Pins of the tanh-layer Rayleigh solver (tests/kh_theory.py) that the
quasi-2D Kelvin-Helmholtz GPU test takes its growth rates from (CPU only).

* The neutral mode: at k = 1 (units of the half-width d) c = 0 and
  phi = sech(y) solve Rayleigh's equation for U = tanh(y) exactly
  (sech'' - sech = -2 sech^3 and U'' = -2 tanh sech^2), so the discretised
  operator annihilates sech, and the growth rate vanishes as k -> 1.
* The long-wave limit: as k -> 0 the layer acts as a vortex sheet between
  -U0 and U0, whose wave speed is c = i U0; Im c extrapolated linearly from
  k = 0.02 and 0.05 reaches 1.
* The fastest-growing mode of the tanh layer (Michalke 1964, J. Fluid Mech.
  19, 543): k d = 0.4446 with sigma d / U0 = 0.1897.
* Convergence in the number of collocation points.
"""
import numpy as np
import pytest

from tests import kh_theory as K


def test_neutral_mode_at_unit_wavenumber():
    xi, D = K._cheb(160)
    xi, D = xi[1:-1], D[1:-1, 1:-1]
    s = np.sqrt(1.0 - xi * xi)
    L = 2.0
    y = L * xi / s
    Dy = (s ** 3 / L)[:, None] * D
    D2 = Dy @ Dy
    U = np.tanh(y)
    Upp = -2.0 * U * (1.0 - U * U)
    phi = 1.0 / np.cosh(y)
    resid = U * ((D2 - np.eye(len(y))) @ phi) - Upp * phi
    assert np.max(np.abs(resid)) <= 1e-8
    assert K.growth_rate(0.995) < 0.01 and K.growth_rate(0.9) > 0.05


def test_long_wave_limit_is_the_vortex_sheet():
    ci = []
    for k in (0.02, 0.05):
        c = K.wave_speeds(k, n=400, L=20.0)
        ci.append(np.max(c[np.isfinite(c)].imag))
    c0 = ci[0] - (ci[1] - ci[0]) / (0.05 - 0.02) * 0.02
    assert abs(c0 - 1.0) <= 5e-3


def test_fastest_growing_mode_matches_the_literature():
    ks = np.linspace(0.40, 0.49, 10)
    s = [K.growth_rate(k) for k in ks]
    assert abs(K.growth_rate(0.4446) - 0.1897) <= 5e-4
    assert abs(ks[int(np.argmax(s))] - 0.4446) <= 0.011


@pytest.mark.parametrize("k", [0.2223, 0.4446, 0.6669])
def test_converged_in_the_collocation_points(k):
    assert abs(K.growth_rate(k, 160) - K.growth_rate(k, 240)) <= 1e-8


@pytest.mark.parametrize("k", [0.2223, 0.6669])
def test_viscous_rates_reduce_to_rayleigh_and_converge(k):
    """The Orr-Sommerfeld rate the GPU test uses: it tends to the (pinned)
    inviscid rate as Re grows, decreases as viscosity rises, and is
    converged in the collocation points at the test's Re."""
    inv = K.growth_rate(k)
    assert abs(K.viscous_growth_rate(k, 1e7) - inv) <= 1e-5 * inv  # an O(1 / Re) correction
    rates = [K.viscous_growth_rate(k, re) for re in (300.0, 1000.0, 2223.0, 1e5)]
    assert all(a < b for a, b in zip(rates, rates[1:])) and rates[-1] < inv
    assert abs(K.viscous_growth_rate(k, 2223.0, 160) - K.viscous_growth_rate(k, 2223.0, 240)) <= 1e-8
