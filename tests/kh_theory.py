"""Linear theory of the Kelvin-Helmholtz instability of a tanh shear layer,
written for the tests (not part of the library or the oracle).

For a parallel inviscid flow U(y), a perturbation stream function
phi(y) exp(i k (x - c t)) obeys Rayleigh's equation

    (U - c) (phi'' - k^2 phi) - U'' phi = 0,

and grows at the temporal rate sigma = k Im(c).  For U = tanh(y) (lengths in
units of the layer half-width d, velocities in units of U0, so sigma is in
units of U0 / d) the equation is discretised by Chebyshev collocation on the
whole line, y = L xi / sqrt(1 - xi^2) with xi in (-1, 1) and phi = 0 at
xi = +-1 (y = +-infinity), which gives the generalised eigenproblem

    [diag(U) (D2 - k^2) - diag(U'')] phi = c (D2 - k^2) phi;

the unstable mode is the eigenvalue of largest imaginary part.
"""
import numpy as np
import scipy.linalg


def _cheb(n):
    """Chebyshev-Gauss-Lobatto points x_j = cos(pi j / n) and the
    differentiation matrix on them (Trefethen, Spectral Methods in MATLAB)."""
    j = np.arange(n + 1)
    x = np.cos(np.pi * j / n)
    c = np.where((j == 0) | (j == n), 2.0, 1.0) * (-1.0) ** j
    X = x[:, None] - x[None, :]
    D = np.outer(c, 1.0 / c) / (X + np.eye(n + 1))
    D -= np.diag(D.sum(axis=1))
    return x, D


def wave_speeds(k: float, n: int = 160, L: float = 2.0) -> np.ndarray:
    """All eigenvalues c of the discretised Rayleigh equation at wavenumber k."""
    xi, D = _cheb(n)
    xi, D = xi[1:-1], D[1:-1, 1:-1]  # phi = 0 at y = +-infinity
    s = np.sqrt(1.0 - xi * xi)
    y = L * xi / s
    dxi_dy = s ** 3 / L
    Dy = dxi_dy[:, None] * D
    # full second derivative: d/dy (dxi/dy d/dxi) with the interior rows of D
    # applied to the interior values (phi vanishes at the ends)
    D2 = Dy @ Dy
    U = np.tanh(y)
    Upp = -2.0 * U * (1.0 - U * U)
    K = D2 - k * k * np.eye(len(y))
    A = U[:, None] * K - np.diag(Upp)
    return scipy.linalg.eigvals(A, K)


def growth_rate(k: float, n: int = 160) -> float:
    """Temporal growth rate sigma = k max Im(c) (units U0 / d) at wavenumber k d."""
    c = wave_speeds(k, n)
    c = c[np.isfinite(c)]
    return float(k * np.max(c.imag))


def viscous_wave_speeds(k: float, re: float, n: int = 160, L: float = 2.0) -> np.ndarray:
    """Eigenvalues c of the Orr-Sommerfeld equation for U = tanh(y) at
    wavenumber k and Reynolds number re = U0 d / nu,

        (U - c) (D2 - k^2) phi - U'' phi = (D2 - k^2)^2 phi / (i k re),

    on the same mapped collocation grid, phi = 0 at y = +-infinity (the
    decaying eigenfunctions also have vanishing derivatives there, which
    the algebraic map imposes to all orders)."""
    xi, D = _cheb(n)
    xi, D = xi[1:-1], D[1:-1, 1:-1]
    s = np.sqrt(1.0 - xi * xi)
    y = L * xi / s
    Dy = (s ** 3 / L)[:, None] * D
    D2 = Dy @ Dy
    U = np.tanh(y)
    Upp = -2.0 * U * (1.0 - U * U)
    K = D2 - k * k * np.eye(len(y))
    A = U[:, None] * K - np.diag(Upp) - (K @ K) / (1j * k * re)
    return scipy.linalg.eigvals(A, K)


def viscous_growth_rate(k: float, re: float, n: int = 160) -> float:
    """Temporal growth rate k Im(c) (units U0 / d) of the Orr-Sommerfeld
    mode that continues the inviscid unstable mode (the eigenvalue nearest
    to it)."""
    c0 = wave_speeds(k, n)
    c0 = c0[np.isfinite(c0)]
    ci = c0[np.argmax(c0.imag)]
    c = viscous_wave_speeds(k, re, n)
    c = c[np.isfinite(c)]
    return float(k * c[np.argmin(np.abs(c - ci))].imag)


def unstable_mode(k: float, n: int = 200, L: float = 2.0):
    """The unstable Rayleigh mode at wavenumber k: its wave speed c, the
    collocation points y (increasing) and phi, phi' there, normalised to
    max |phi| = 1 (stream function phi(y) exp(i k x))."""
    xi, D = _cheb(n)
    xi, D = xi[1:-1], D[1:-1, 1:-1]
    s = np.sqrt(1.0 - xi * xi)
    y = L * xi / s
    Dy = (s ** 3 / L)[:, None] * D
    D2 = Dy @ Dy
    U = np.tanh(y)
    Upp = -2.0 * U * (1.0 - U * U)
    K = D2 - k * k * np.eye(len(y))
    A = U[:, None] * K - np.diag(Upp)
    w, V = scipy.linalg.eig(A, K)
    w = np.where(np.isfinite(w), w, 0.0)
    j = int(np.argmax(w.imag))
    phi = V[:, j] / V[np.argmax(np.abs(V[:, j])), j]
    dphi = Dy @ phi
    order = np.argsort(y)
    return w[j], y[order], phi[order], dphi[order]
