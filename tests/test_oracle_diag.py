"""Pins of the oracle diagnostics: the compensated sum against math.fsum, the
spectral (Parseval) quantities against real-space means computed another way
(numpy FFTs), and closed-form values for analytic states."""
import math

import numpy as np

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I


def test_neumaier_matches_fsum():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 1e-3, [1e16, 1.0, -1e16, 3.0]])
    rng.shuffle(x)
    exact = math.fsum(x)
    # Neumaier's bound: |err| <= 2u|S| + O(n u^2) sum|x_i|
    u = 2.0 ** -53
    bound = 2 * u * abs(exact) + 4 * x.size * u * u * np.abs(x).sum()
    assert abs(O.neumaier_sum(x) - exact) <= bound
    naive = 0.0
    for v in x:
        naive += v
    assert abs(naive - exact) > 100 * bound  # the cancellation defeats plain summation


def test_abc_closed_form_energies():
    c = I.config_small(16)
    d = O.diag(c.U, c.gamma, c.nu, c.eta)
    # ABC with A = B = C = 1: <|u|^2> = 3, rho = 1 -> E_K = 3/2; P = 60 -> E_I = 90
    assert abs(d["e_kin"] - 1.5) < 1e-13
    assert abs(d["e_int"] - 90.0) < 1e-11
    assert abs(d["mass"] - 1.0) < 1e-15
    assert abs(d["c_s"] - 10.0) < 1e-12
    assert abs(d["e_mag"] - 0.5e-6) < 1e-15  # rms |B| = 1e-3
    assert d["divb_rel"] < 1e-13


def test_spectral_diagnostics_against_real_space():
    n = 16
    c = I.random_turbulence(n, seeds=(3, 4, 5), b_rms=0.3)
    U = c.U.copy()
    # add a compressive part to B so that div B is nonzero and measurable
    z, y, x = I.grid(n)
    U[4] += 0.05 * np.sin(2 * x + y)
    d = O.diag(U, c.gamma, c.nu, c.eta)
    B = np.stack([O.project(U[4 + i]) for i in range(3)])
    Bh = np.fft.fftn(B, axes=(1, 2, 3))
    k = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    Kv = np.stack([KX, KY, KZ])
    K2 = np.where(KX ** 2 + KY ** 2 + KZ ** 2 == 0, 1.0, KX ** 2 + KY ** 2 + KZ ** 2)
    Jh = 1j * np.cross(Kv, Bh, axis=0)
    Ah = Jh / K2
    A = np.real(np.fft.ifftn(Ah, axes=(1, 2, 3)))
    J = np.real(np.fft.ifftn(Jh, axes=(1, 2, 3)))
    divb = np.real(np.fft.ifftn(1j * np.sum(Kv * Bh, axis=0)))
    assert abs(d["h_mag"] - np.mean(np.sum(A * B, axis=0))) < 1e-13 * max(1.0, abs(d["h_mag"]))
    assert abs(d["divb_rms"] - np.sqrt(np.mean(divb ** 2))) < 1e-13
    assert abs(d["divb_max"] - np.abs(divb).max()) < 1e-13
    assert abs(d["j_rms"] - np.sqrt(np.mean(np.sum(J * J, axis=0)))) < 1e-12
    assert d["divb_rms"] > 1e-3


def test_force_free_helicity_and_cfl():
    """B = B0 (sin z, cos z, 0) is its own curl (J = B), so A = B and
    H_M = <|B|^2> = B0^2; c_f and the CFL step follow in closed form."""
    n, B0, rho0, P0, gamma = 8, 0.8, 1.2, 1.5, 5.0 / 3.0
    z, y, x = I.grid(n)
    B = np.zeros((3, n, n, n))
    B[0] = B0 * np.sin(z) + 0 * x + 0 * y
    B[1] = B0 * np.cos(z) + 0 * x + 0 * y
    U = I.conserved(np.full((n, n, n), rho0), np.zeros((3, n, n, n)), B, np.full((n, n, n), P0), gamma)
    d = O.diag(U, gamma, cfl=0.2)
    assert abs(d["h_mag"] - B0 ** 2) < 1e-14
    cf = math.sqrt((gamma * P0 + B0 ** 2) / rho0)
    assert abs(d["dt_cfl"] - 0.2 * (2 * math.pi / n) / cf) < 1e-14
    assert abs(d["v_a"] - B0 / math.sqrt(rho0)) < 1e-14
    assert d["nonfinite"] == 0


def test_nonfinite_count():
    c = I.config_small(8)
    U = c.U.copy()
    U[3, 1, 2, 3] = np.nan
    U[7, 0, 0, 0] = np.inf
    assert O.diag(U, c.gamma)["nonfinite"] == 2


def _cp_wave_diag(rho0, b0, B0=1.0, P0=0.7, n=12, axis=2):
    from tests.test_oracle_rhs import cp_alfven

    U = cp_alfven(n, 0.0, axis=axis, k=1, B0=B0, b0=b0, rho0=rho0, P0=P0)
    return U, O.diag(U, 5.0 / 3.0)


def test_cross_helicity_closed_form_varying_density():
    """Circularly polarised Alfven wave with rho0 != 1: u_perp = -b_perp / sqrt(rho0)
    and B = B0 e_axis + b_perp, so u.B = -b0^2 / sqrt(rho0) at every point (paper
    Section V-B reads the cross term u.B).  Using m.B instead of u.B would give
    -sqrt(rho0) b0^2, 2.25x larger in magnitude at rho0 = 2.25."""
    rho0, b0 = 2.25, 0.4
    _, d = _cp_wave_diag(rho0, b0)
    assert abs(d["h_cross"] - (-b0 * b0 / math.sqrt(rho0))) < 1e-14
    assert abs(d["h_cross"] - (-math.sqrt(rho0) * b0 * b0)) > 0.1


def test_mach_numbers_closed_form():
    """Section III: c_s = sqrt(gamma <P>/<rho>), V_A = <|B|>/sqrt(<rho>),
    M_s = <|u|>/c_s, M_A = <|u|>/V_A.  On the CP wave |u| = b0/sqrt(rho0) and
    |B| = sqrt(B0^2 + b0^2) at every point, P = P0 and rho = rho0."""
    gamma, rho0, b0, B0, P0 = 5.0 / 3.0, 2.25, 0.4, 1.3, 0.7
    _, d = _cp_wave_diag(rho0, b0, B0=B0, P0=P0)
    cs = math.sqrt(gamma * P0 / rho0)
    va = math.sqrt(B0 * B0 + b0 * b0) / math.sqrt(rho0)
    uabs = b0 / math.sqrt(rho0)
    assert abs(d["c_s"] - cs) < 1e-14
    assert abs(d["v_a"] - va) < 1e-14
    assert abs(d["mach_s"] - uabs / cs) < 1e-14
    assert abs(d["mach_a"] - uabs / va) < 1e-14
    # a <|m|> numerator (rho0 times larger) or a missing sqrt in V_A would miss
    assert abs(d["mach_s"] - rho0 * uabs / cs) > 0.1 * uabs / cs
    assert abs(d["v_a"] - math.sqrt(B0 * B0 + b0 * b0) / rho0) > 0.1 * va


def test_cross_helicity_conserved_isentropic_ideal():
    """Ideal MHD conserves <u.B> when the pressure is a function of density
    alone; an isentropic start P = K rho^gamma stays isentropic while the flow is
    smooth, so the only drift of the discrete run is the integrator's O(dt^2).
    Halving dt must cut the drift about 4x (and H_M and E_tot stay put)."""
    gamma, n, T = 5.0 / 3.0, 16, 0.06
    z, y, x = I.grid(n)
    rho = 1.0 + 0.2 * np.cos(x + y) + 0.1 * np.sin(z) + 0 * x
    u = np.zeros((3, n, n, n))
    u[0] = 0.4 * np.sin(y) + 0.2 * np.cos(z) + 0 * x
    u[1] = 0.3 * np.sin(z) + 0.2 * np.cos(x) + 0 * y
    u[2] = 0.3 * np.sin(x + y) + 0 * z
    B = np.zeros((3, n, n, n))
    B[0] = 0.5 * np.cos(y + z) + 0.2 + 0 * x
    B[1] = 0.4 * np.sin(z) + 0.3 * np.cos(x) + 0 * y
    B[2] = 0.3 * np.sin(x - y) + 0.1 + 0 * z
    P = 1.5 * rho ** gamma
    U0 = I.conserved(rho, u, B, P, gamma)
    d0 = O.diag(U0, gamma)
    assert abs(d0["h_cross"]) > 0.01
    drift = []
    for steps in (60, 120, 240):
        U = O.run(U0, steps, T / steps, gamma)
        d1 = O.diag(U, gamma)
        assert abs(d1["e_tot"] - d0["e_tot"]) < 1e-12 * d0["e_tot"]
        drift.append(abs(d1["h_cross"] - d0["h_cross"]))
    r1, r2 = drift[0] / drift[1], drift[1] / drift[2]
    assert 3.2 < r1 < 4.8 and 3.2 < r2 < 4.8, drift
