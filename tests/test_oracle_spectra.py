"""Pins of the oracle's Section V turbulence diagnostics against closed forms:
shell spectra of single Fourier modes, the rms velocity divergence theta' and
the skewness S_3 of du_x/dx, and the k^4 exp(-2k^2/k0^2) start.

* B = b cos(k0.x) puts b^2/4 (= <|B|^2>/2) in shell floor(|k0| + 1/2) and
  nothing elsewhere; u = a sin(2x) x + c cos(3y) y (rho = 1) puts a^2/4 and
  c^2/4 in shells 2 and 3.
* theta' of that u: div u = 2a cos 2x - 3c sin 3y, so theta' = (2a^2 + 9c^2/2)^(1/2);
  du_x/dx alone has rms sqrt(2) a.
* u_x = sin x + a sin 2x: d = cos x + 2a cos 2x, <d^3> = 3(2a)/4,
  <d^2> = (1 + 4a^2)/2, so S_3 = (3a/2) / ((1 + 4a^2)/2)^(3/2).
* The decaying-turbulence start's shell spectrum follows k^4 exp(-2k^2/k0^2)
  (ratios of shell sums over neighbouring shells, within sampling noise) and
  it is solenoidal.
"""
import numpy as np

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I


def state(n, u=None, B=None, rho=None, P=0.7, gamma=5.0 / 3.0):
    z, y, x = I.grid(n)
    zero = np.zeros((3, n, n, n))
    return I.conserved(np.ones((n, n, n)) if rho is None else rho, zero if u is None else u,
                       zero if B is None else B, np.full((n, n, n), P), gamma)


def test_single_mode_spectra_and_moments():
    n = 16
    z, y, x = I.grid(n)
    b, a, c = 0.6, 0.3, 0.2
    B = np.zeros((3, n, n, n))
    B[2] = b * np.cos(1 * x + 2 * y + 0 * z)  # |k| = sqrt(5) -> shell 2 (k . B = 0: solenoidal)
    u = np.zeros((3, n, n, n))
    u[0] = a * np.sin(2 * x) + 0 * (y + z)
    u[1] = c * np.cos(3 * y) + 0 * (x + z)
    s = O.spectra(state(n, u, B), 8)
    want_b = np.zeros(8)
    want_b[2] = b * b / 4
    want_u = np.zeros(8)
    want_u[2], want_u[3] = a * a / 4, c * c / 4
    assert np.abs(s["e_b"] - want_b).max() < 1e-15
    assert np.abs(s["e_u"] - want_u).max() < 1e-15
    # div u = 2a cos 2x - 3c sin 3y
    assert abs(s["theta_rms"] - np.sqrt(2 * a * a + 4.5 * c * c)) < 1e-14
    assert abs(s["dudx_rms"] - np.sqrt(2) * a) < 1e-14


def test_skewness_closed_form():
    n, a = 16, 0.35
    z, y, x = I.grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(x) + a * np.sin(2 * x) + 0 * (y + z)
    s = O.spectra(state(n, u), 8)
    want = (1.5 * a) / ((1 + 4 * a * a) / 2) ** 1.5
    assert abs(s["s3"] - want) < 1e-13
    # the sign follows the asymmetry of the gradient distribution
    u[0] = np.sin(x) - a * np.sin(2 * x) + 0 * (y + z)
    assert abs(O.spectra(state(n, u), 8)["s3"] + want) < 1e-13


def test_magnetic_spectrum_sums_to_the_magnetic_energy():
    c = I.random_turbulence(24, b_rms=0.4, seeds=(3, 4, 5))
    s = O.spectra(c.U, 40)
    assert abs(s["e_b"].sum() - O.diag(c.U, c.gamma)["e_mag"]) < 1e-14 * s["e_b"].sum()


def test_k4_start_spectrum_shape():
    n, k0 = 48, 4.0
    c = I.decaying_turbulence(n, k0=k0)
    u = c.U[1:4] / c.U[0]
    assert abs(np.sqrt(np.mean(np.sum(u * u, axis=0))) - 1.0) < 1e-12
    s = O.spectra(c.U, 16)["e_u"]
    E = lambda k: k ** 4 * np.exp(-2 * k * k / (k0 * k0))  # noqa: E731
    # shell sums of a Gaussian field: ratio to the model, normalised, within sampling noise
    shells = np.arange(2, 11)
    r = s[shells] / E(shells.astype(float))
    r /= np.median(r)
    assert np.all(np.abs(r - 1) < 0.35), r
    assert s[1:].argmax() + 1 in (int(k0) - 1, int(k0), int(k0) + 1)
    k = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    div = sum(np.fft.fftn(u[i]) * kk for i, kk in enumerate((kx, ky, kz)))
    assert np.abs(div).max() < 1e-9 * np.abs(np.fft.fftn(u[0])).max()
