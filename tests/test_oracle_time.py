"""Pins of the oracle's time integrator and conservation properties.

* Force-free helical field B = B0 (sin z, cos z, 0), u = 0: the induction RHS
  is exactly -eta B, every other RHS vanishes, so the discrete solution is the
  AB2 recurrence y1 = (1+z) y0, y_{n+1} = (1 + 3z/2) y_n - (z/2) y_{n-1},
  z = -eta dt.  This fixes the coefficients and the Euler start.
* Second-order convergence on the exact decaying circularly polarised wave.
* Mass, momentum and total energy are conserved to roundoff for any nu, eta
  (divergence form), and div B stays at roundoff.
"""
import numpy as np

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I
from tests.test_oracle_rhs import GAMMA, cp_alfven


def force_free(n, B0=0.8, rho0=1.2, P0=1.5):
    z, y, x = I.grid(n)
    B = np.zeros((3, n, n, n))
    B[0] = B0 * np.sin(z) + 0 * x + 0 * y
    B[1] = B0 * np.cos(z) + 0 * x + 0 * y
    u = np.zeros((3, n, n, n))
    return I.conserved(np.full((n, n, n), rho0), u, B, np.full((n, n, n), P0), GAMMA)


def test_ab2_recurrence_force_free():
    n, eta, dt, steps = 8, 0.07, 0.05, 20
    U0 = force_free(n)
    U = O.run(U0, steps, dt, GAMMA, nu=0.01, eta=eta)
    zc = -eta * dt
    y_prev, y = 1.0, 1.0 + zc
    for _ in range(steps - 1):
        y_prev, y = y, (1 + 1.5 * zc) * y - 0.5 * zc * y_prev
    assert np.abs(U[4:7] - y * U0[4:7]).max() < 1e-13
    assert np.abs(U[1:4]).max() < 1e-13
    assert np.abs(U[7] - U0[7]).max() < 1e-12
    # a different integrator (plain Euler, or AB2 without the Euler start) misses
    assert abs(y - (1 + zc) ** steps) > 1e-6


def test_second_order_convergence():
    n, nu, T = 8, 0.05, 0.4
    errs = []
    for steps in (40, 80, 160):
        U = O.run(cp_alfven(n, 0.0, axis=1, k=1, nu=nu), steps, T / steps, GAMMA, nu=nu, eta=nu)
        exact = cp_alfven(n, T, axis=1, k=1, nu=nu)
        errs.append(np.abs(U - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_conservation_and_divb():
    c = I.random_turbulence(16, nu=5e-3, eta=8e-3, seeds=(11, 12, 13))
    d0 = O.diag(c.U, c.gamma, c.nu, c.eta)
    U = O.run(c.U, 20, c.dt, c.gamma, c.nu, c.eta)
    d1 = O.diag(U, c.gamma, c.nu, c.eta)
    assert abs(d1["mass"] - d0["mass"]) < 1e-14
    for k in ("mom_x", "mom_y", "mom_z"):
        assert abs(d1[k] - d0[k]) < 1e-14
    assert abs(d1["e_tot"] - d0["e_tot"]) < 1e-13 * d0["e_tot"]
    assert d1["divb_rel"] < 1e-13
    # the run did something: kinetic energy changed
    assert abs(d1["e_kin"] - d0["e_kin"]) > 1e-6


def test_ideal_limit_energy_exchange():
    """Ideal limit: the kinetic + magnetic + internal split moves while the total
    stays fixed, and magnetic helicity drifts only at O(dt^2)."""
    c = I.abc_dynamo(16, nu=0.0, eta=0.0, dt=2e-3, b_rms=0.3, seed=21)
    d0 = O.diag(c.U, c.gamma)
    drift = []
    for dt in (2e-3, 1e-3):
        U = O.run(c.U, int(round(0.04 / dt)), dt, c.gamma)
        d1 = O.diag(U, c.gamma)
        assert abs(d1["e_tot"] - d0["e_tot"]) < 1e-12 * d0["e_tot"]
        drift.append(abs(d1["h_mag"] - d0["h_mag"]))
    assert drift[1] < drift[0] / 2.5 or drift[0] < 1e-12
