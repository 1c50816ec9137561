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
