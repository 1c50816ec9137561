"""Quasi-2D Kelvin-Helmholtz run (the paper's Section IV shear-layer test) on
the GPU, against the linear theory of the tanh shear layer.

The paper's runs start from tanh shear layers (vorticity omega0 sech^2 of
the distance to the layer over d) and compare the growth rates of single
modes with a closed form (Drazin's).  As printed, that formula cannot be
pinned (its variables are not made dimensionless consistently, it describes
a broken-line profile rather than the tanh layers the runs start from, and
it is stated for twice the growth rate), so the growth rates here are held
to the linear theory of the tanh layer itself: the Orr-Sommerfeld equation
at the run's Reynolds number, solved in tests/kh_theory.py (whose inviscid
limit, Rayleigh's equation, tests/test_kh_theory.py pins to its neutral and
long-wave closed forms and to the tabulated fastest mode).

Set-up: 256^3 with every field independent of z (quasi-2D), two layers
u_x = U0 [tanh((y - pi/2)/d) - tanh((y - 3pi/2)/d) - 1], d = 0.2223, so the
modes k = 1, 2, 3 of the 2 pi box sit at k d = 0.22, 0.44 (the fastest
growing) and 0.67; rho = 1, sound speed 10 U0 (Mach 0.1), nu = 1e-4
(U0 d / nu = 2223), B = 0.  Each mode is seeded at the lower layer with its
own linear eigenfunction (amplitude 1e-5 U0), so the mode grows from the
start without a transient; the amplitude of mode k of u_y must grow as
exp(sigma_k t) with sigma_k the Orr-Sommerfeld rate within 3% (what the
theory leaves out: compressibility at Mach 0.1, about 1%, and the slow
diffusion of the base flow over the run, 4 nu t / d^2 = 0.03).  The grid
must resolve the eigenfunctions: an unstable tanh mode has a complex
critical point Im(c) d off the real axis (0.23 d at k d = 0.67), so its
spectrum decays like exp(-0.23 d k_y); at 128^3 that is 0.12 at the
dealiasing cutoff and the k d = 0.67 rate came out 4.5% low, at 256^3 it is
0.013.  FP32 only (the benchmark path); at 128^3 FP32 and FP64 gave the
same rates to 0.3%.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from tests.gpu_helpers import log
from tests.kh_theory import unstable_mode, viscous_growth_rate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, D, U0, CS, NU, GAMMA = 256, 0.2223, 1.0, 10.0, 1e-4, 5.0 / 3.0
MODES = (1, 2, 3)
EPS = 1e-5


def kh_state(n, dtype):
    xs = np.arange(n) * (2 * math.pi / n)
    x, y = xs[None, :], xs[:, None]  # [y][x] plane, the same on every z
    ux = U0 * (np.tanh((y - math.pi / 2) / D) - np.tanh((y - 3 * math.pi / 2) / D) - 1.0) + 0 * x
    uy = np.zeros((n, n))
    eta = (xs - math.pi / 2) / D
    for k in MODES:
        _, yc, phi, dphi = unstable_mode(k * D)
        p = CubicSpline(yc, phi.real)(eta) + 1j * CubicSpline(yc, phi.imag)(eta)
        dp = CubicSpline(yc, dphi.real)(eta) + 1j * CubicSpline(yc, dphi.imag)(eta)
        e = np.exp(1j * k * xs)[None, :]
        # stream function EPS U0 d phi(eta) e^{ikx}: u_x = d psi/dy, u_y = -d psi/dx
        ux = ux + EPS * U0 * np.real(dp[:, None] * e)
        uy = uy + EPS * U0 * np.real(-1j * k * D * p[:, None] * e)
    rho = 1.0
    P = rho * CS * CS / GAMMA
    U = torch.zeros((8, n, n, n), dtype=dtype, device="cuda:0")
    U[0] = rho
    U[1] = torch.from_numpy(rho * ux).to(device="cuda:0", dtype=dtype)[None]
    U[2] = torch.from_numpy(rho * uy).to(device="cuda:0", dtype=dtype)[None]
    U[7] = torch.from_numpy(P / (GAMMA - 1.0) + 0.5 * rho * (ux * ux + uy * uy)).to(device="cuda:0",
                                                                                    dtype=dtype)[None]
    return U


def mode_amplitudes(S, n):
    """rms over y of |(1/n) sum_x u_y e^{-i k x}| at z = 0, for each seeded k."""
    st = S.get_state(torch.float64)
    uy = (st[2, 0] / st[0, 0])  # [y][x]
    del st
    xs = torch.arange(n, dtype=torch.float64, device="cuda:0") * (2 * math.pi / n)
    out = []
    for k in MODES:
        e = torch.exp(-1j * k * xs).to(torch.complex128)
        a = (uy.to(torch.complex128) @ e) / n
        out.append(float(torch.sqrt(torch.mean(torch.abs(a) ** 2))))
    return out


def test_kelvin_helmholtz_growth_rates():
    from paper_1810_12707_amd.mhd import Solver

    # AB2 amplifies a purely oscillatory mode by about 1 + (lambda dt)^4 / 4 per
    # step; the fastest acoustic mode (k = 85, sound speed 10) has
    # lambda dt = 0.10 here, so rounding noise grows by ~2 over the run
    # (at 128^3 with lambda dt = 0.34 it grew by e^25 and the run went
    # non-finite)
    prec = "fp32"
    dt = 1.2e-4
    chunk, nchunks = 1000, 32  # t = 3.84
    log(f"[kh] n={N} prec={prec} dt={dt} steps={chunk * nchunks}")
    S = Solver(N, precision=prec, gamma=GAMMA, nu=NU, eta=NU, dt=dt)
    S.set_state(kh_state(N, torch.float32))
    t, amps = [0.0], [mode_amplitudes(S, N)]
    for c in range(nchunks):
        S.step(chunk)
        t.append((c + 1) * chunk * dt)
        amps.append(mode_amplitudes(S, N))
    rc, _ = S.diagnostics()
    S.close()
    assert rc == 0
    t, amps = np.array(t), np.array(amps)
    fit = t >= 0.5
    re = U0 * D / NU
    for j, k in enumerate(MODES):
        slope = np.polyfit(t[fit], np.log(amps[fit, j]), 1)[0]
        early = np.polyfit(t[fit][:10], np.log(amps[fit, j][:10]), 1)[0]  # drifts with the base flow
        want = viscous_growth_rate(k * D, re) * U0 / D
        log(f"  k={k} (kd={k * D:.3f}): growth {slope:.4f} (first third {early:.4f}), Orr-Sommerfeld {want:.4f}, "
            f"ratio {slope / want:.4f}, amplitude {amps[0, j]:.2e} -> {amps[-1, j]:.2e}")
        assert abs(slope / want - 1.0) <= 0.03
        assert amps[-1, j] < 0.02 * U0  # still linear
