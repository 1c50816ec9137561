"""Pins of the oracle's other time integrators (Runge-Kutta 4 and the
Adams-Bashforth-Moulton predictor-corrector; Section II names both beside
Adams-Bashforth) and of the Section V variants (viscous force nu lap u, the
ABC body force, the kinematic mode), against closed forms.

* Force-free helical field B = B0 (sin z, cos z, 0), u = 0: the induction RHS
  is exactly -eta B and every other field's evolution is fixed by it, so each
  integrator reduces to its scalar recurrence on y' = -eta y: RK4 multiplies by
  1 + z + z^2/2 + z^3/6 + z^4/24 per step (z = -eta dt); the predictor-
  corrector runs y* = y_n + z (3/2 y_n - 1/2 y_{n-1}) (Euler first),
  y_{n+1} = y_n + z/2 (y_n + y*).  This fixes every coefficient and the start.
* Order: on the exact decaying circularly polarised Alfven wave the RK4 error
  falls 16x and the predictor-corrector's 4x per halving of dt.
* The three integrators agree on a turbulent start to O(dt^2).
* nu lap u: on u = (sin x, 0, 0), rho = 1, the k = 1 momentum RHS is -nu sin x
  (the stress form gives -4/3 nu sin x), and the energy gains
  nu lap(|u|^2/2) = nu cos 2x.
* ABC force: the change of the RHS is rho f in m and m.f in E, exactly, for a
  state where these products are trigonometric polynomials inside the band.
* Kinematic mode: rho, m and E have zero RHS, and B's RHS is unchanged.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I
from tests.test_oracle_rhs import GAMMA, cp_alfven
from tests.test_oracle_time import force_free


def rk4_factor(zc):
    return 1 + zc + zc ** 2 / 2 + zc ** 3 / 6 + zc ** 4 / 24


def pc_sequence(zc, steps):
    y_prev, y = 1.0, 1.0
    for s in range(steps):
        if s == 0:
            ys = y + zc * y  # Euler predictor on the first step
        else:
            ys = y + zc * (1.5 * y - 0.5 * y_prev)
        y_prev, y = y, y + 0.5 * zc * (y + ys)
    return y


@pytest.mark.parametrize("scheme", ["rk4", "pc"])
def test_recurrence_force_free(scheme):
    n, eta, dt, steps = 8, 0.07, 0.05, 20
    U0 = force_free(n)
    U = O.run(U0, steps, dt, GAMMA, nu=0.01, eta=eta, scheme=scheme)
    zc = -eta * dt
    y = rk4_factor(zc) ** steps if scheme == "rk4" else pc_sequence(zc, steps)
    assert np.abs(U[4:7] - y * U0[4:7]).max() < 1e-13
    assert np.abs(U[1:4]).max() < 1e-13
    assert np.abs(U[7] - U0[7]).max() < 1e-12
    # the other recurrences miss by far more than rounding
    other = pc_sequence(zc, steps) if scheme == "rk4" else rk4_factor(zc) ** steps
    assert abs(y - other) > 1e-9
    ab2_prev, ab2 = 1.0, 1.0 + zc
    for _ in range(steps - 1):
        ab2_prev, ab2 = ab2, (1 + 1.5 * zc) * ab2 - 0.5 * zc * ab2_prev
    assert abs(y - ab2) > 1e-9


@pytest.mark.parametrize("scheme,ratio", [("rk4", 16.0), ("pc", 4.0)])
def test_order_on_the_exact_alfven_wave(scheme, ratio):
    n, nu, T = 8, 0.05, 0.4
    errs = []
    for steps in ((5, 10, 20) if scheme == "rk4" else (40, 80, 160)):
        U = O.run(cp_alfven(n, 0.0, axis=2, k=1, nu=nu), steps, T / steps, GAMMA, nu=nu, eta=nu, scheme=scheme)
        errs.append(np.abs(U - cp_alfven(n, T, axis=2, k=1, nu=nu)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 0.85 * ratio < r1 < 1.15 * ratio and 0.85 * ratio < r2 < 1.15 * ratio, errs


def test_integrators_agree_at_second_order():
    c = I.random_turbulence(16, nu=5e-3, eta=8e-3, seeds=(11, 12, 13))
    T = 0.04
    diffs = {}
    for steps in (10, 20):
        dt = T / steps
        runs = {s: O.run(c.U, steps, dt, c.gamma, c.nu, c.eta, scheme=s) for s in ("ab2", "rk4", "pc")}
        scale = np.abs(runs["rk4"]).max()
        diffs[steps] = (np.abs(runs["ab2"] - runs["rk4"]).max() / scale,
                        np.abs(runs["pc"] - runs["rk4"]).max() / scale)
    for i in range(2):
        r = diffs[10][i] / diffs[20][i]
        assert 3.2 < r < 4.8, diffs
        assert diffs[20][i] < 1e-4  # small already: the schemes solve the same equations


def shear_state(n, rho_amp=0.0):
    z, y, x = I.grid(n)
    rho = 1.0 + rho_amp * np.cos(x) + 0 * (y + z)
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(x) + 0 * (y + z)
    B = np.zeros((3, n, n, n))
    P = np.full((n, n, n), 0.9)
    return I.conserved(rho, u, B, P, GAMMA), (z, y, x)


def test_laplacian_viscosity_variant():
    n, nu = 16, 0.03
    U, (z, y, x) = shear_state(n)
    kx1 = lambda f: 2 * np.mean(f * np.sin(x + 0 * (y + z)))  # noqa: E731  sin x coefficient
    R_lap = O.rhs(U, GAMMA, nu, 0.0, options=O.VISC_LAPLACIAN)
    R_str = O.rhs(U, GAMMA, nu, 0.0)
    R_0 = O.rhs(U, GAMMA, 0.0, 0.0)
    assert abs(kx1(R_lap[1] - R_0[1]) - (-nu)) < 1e-13
    assert abs(kx1(R_str[1] - R_0[1]) - (-4.0 / 3.0 * nu)) < 1e-13
    # energy: nu lap(|u|^2/2) = nu cos 2x, and <R_E> = 0
    assert np.abs((R_lap[7] - R_0[7]) - nu * np.cos(2 * x + 0 * (y + z))).max() < 1e-13
    assert abs(np.mean(R_lap[7])) < 1e-14
    # only m and E change
    for f in (0, 2, 3, 4, 5, 6):
        assert np.abs(R_lap[f] - R_0[f]).max() < 1e-14


def test_abc_force():
    n, F0 = 16, 0.35
    U, (z, y, x) = shear_state(n, rho_amp=0.2)
    f = np.stack([np.sin(z) + np.cos(y) + 0 * x, np.sin(x) + np.cos(z) + 0 * y, np.sin(y) + np.cos(x) + 0 * z])
    dR = O.rhs(U, GAMMA, 0.01, 0.02, force=F0) - O.rhs(U, GAMMA, 0.01, 0.02)
    rho, m = U[0], U[1:4]
    for i in range(3):
        assert np.abs(dR[1 + i] - F0 * rho * f[i]).max() < 1e-13
    assert np.abs(dR[7] - F0 * np.sum(m * f, axis=0)).max() < 1e-13
    for k in (0, 4, 5, 6):
        assert np.abs(dR[k]).max() < 1e-14


def test_kinematic_mode():
    c = I.abc_dynamo(16, nu=0.02, eta=0.03, dt=1e-3, b_rms=0.1, seed=5)
    R = O.rhs(c.U, c.gamma, c.nu, c.eta)
    Rk = O.rhs(c.U, c.gamma, c.nu, c.eta, options=O.KINEMATIC)
    for k in (0, 1, 2, 3, 7):
        assert np.abs(Rk[k]).max() == 0.0
    assert np.abs(Rk[4:7] - R[4:7]).max() < 1e-14
    # stepping keeps the flow exactly frozen while B evolves
    U = O.run(c.U, 5, c.dt, c.gamma, c.nu, c.eta, options=O.KINEMATIC)
    P = np.stack([O.project(c.U[k]) for k in (0, 1, 2, 3, 7)])
    assert np.abs(U[[0, 1, 2, 3, 7]] - P).max() < 1e-13
    assert np.abs(U[4:7] - c.U[4:7]).max() > 1e-6
