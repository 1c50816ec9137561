"""Pins of the oracle's full right-hand side against things other than its own
formulas.

1. Exact reduction.  For a state whose primitive variables are trigonometric
   polynomials of degree <= 1 per axis (rho, u, B, P), every flux has degree <= 4,
   so on n = 16 (retained |k| <= 5, products alias-free) the pseudo-spectral RHS
   equals the continuous one.  The continuous time derivatives are derived here
   by sympy from the textbook NON-conservative (primitive-variable) form of
   viscous-resistive ideal-gas MHD:
       d_t rho = -div(rho u)
       rho d_t u = -rho (u.grad) u - grad P + J x B + div(2 nu rho S)
       d_t B = curl(u x B) + eta lap B
       d_t P = -u.grad P - gamma P div u + (gamma-1)(2 nu rho S:S + eta |J|^2)
   and mapped to conserved variables by the chain rule, so a dropped term, a
   wrong sign or a transposed index in the oracle's conservative fluxes fails.
2. Linear waves.  The oracle's linearisation about a uniform magnetised state,
   probed mode by mode, has the textbook eigenvalues: slow, Alfven and fast
   frequencies, and the viscous/resistive damping rates.
3. An exact nonlinear solution (circularly polarised Alfven wave with nu = eta)
   and special cases (uniform state, k = 0 modes, axis permutations).
"""
import numpy as np
import pytest
import sympy as sp

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I

GAMMA = 5.0 / 3.0


# --------------------------------------------------------------------------- #
# 1. exact reduction against the primitive form                               #
# --------------------------------------------------------------------------- #

def _primitive_trig_state(seed):
    """Random degree-1 trigonometric polynomials; B solenoidal by construction
    (each component depends only on the two other coordinates)."""
    rng = np.random.default_rng(seed)
    x, y, z = sp.symbols("x y z", real=True)
    X = (x, y, z)

    def r(scale=1.0):
        return sp.Float(float(rng.uniform(-1, 1) * scale), 17)

    def trig(vars_, scale):
        # sum over a few modes with wavevector entries in {-1, 0, 1}
        expr = 0
        for _ in range(3):
            kv = [int(v) for v in rng.integers(-1, 2, size=len(vars_))]
            arg = sum(k * v for k, v in zip(kv, vars_)) + r(np.pi)
            expr += r(scale) * sp.cos(arg)
        return expr

    rho = 1 + trig(X, 0.1)
    u = [trig(X, 0.5) + r(0.3) for _ in range(3)]
    B = [trig((y, z), 0.5) + r(0.5), trig((z, x), 0.5) + r(0.5), trig((x, y), 0.5) + r(0.5)]
    P = 2 + trig(X, 0.2)
    return X, rho, u, B, P


def _primitive_rhs(X, rho, u, B, P, gamma, nu, eta):
    x, y, z = X
    d = lambda f, j: sp.diff(f, X[j])  # noqa: E731
    div_u = sum(d(u[j], j) for j in range(3))
    grad_u = [[d(u[i], j) for j in range(3)] for i in range(3)]  # grad_u[i][j] = d_j u_i
    S = [[sp.Rational(1, 2) * (grad_u[i][j] + grad_u[j][i]) - (div_u / 3 if i == j else 0)
          for j in range(3)] for i in range(3)]
    J = [d(B[2], 1) - d(B[1], 2), d(B[0], 2) - d(B[2], 0), d(B[1], 0) - d(B[0], 1)]
    JxB = [J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]]
    visc = [sum(d(2 * nu * rho * S[i][j], j) for j in range(3)) for i in range(3)]
    rho_t = -sum(d(rho * u[j], j) for j in range(3))
    rho_ut = [-rho * sum(u[j] * grad_u[i][j] for j in range(3)) - d(P, i) + JxB[i] + visc[i]
              for i in range(3)]
    uxB = [u[1] * B[2] - u[2] * B[1], u[2] * B[0] - u[0] * B[2], u[0] * B[1] - u[1] * B[0]]
    curl = lambda F: [d(F[2], 1) - d(F[1], 2), d(F[0], 2) - d(F[2], 0), d(F[1], 0) - d(F[0], 1)]  # noqa: E731
    lap = lambda f: sum(sp.diff(f, v, 2) for v in X)  # noqa: E731
    B_t = [c + eta * lap(b) for c, b in zip(curl(uxB), B)]
    SS = sum(S[i][j] * S[i][j] for i in range(3) for j in range(3))
    J2 = sum(j * j for j in J)
    P_t = (-sum(u[j] * d(P, j) for j in range(3)) - gamma * P * div_u
           + (gamma - 1) * (2 * nu * rho * SS + eta * J2))
    u2 = sum(c * c for c in u)
    m_t = [rho_ut[i] + u[i] * rho_t for i in range(3)]
    E_t = (P_t / (gamma - 1) + u2 / 2 * rho_t + sum(u[i] * rho_ut[i] for i in range(3))
           + sum(B[i] * B_t[i] for i in range(3)))
    return [rho_t] + m_t + B_t + [E_t]


def _evaluate(exprs, X, n):
    z, y, x = I.grid(n)
    shape = (n, n, n)
    out = []
    for e in exprs:
        f = sp.lambdify(X, e, "numpy")
        v = np.broadcast_to(np.asarray(f(x, y, z), dtype=np.float64), shape)
        out.append(np.array(v))
    return np.stack(out)


@pytest.mark.parametrize("seed,nu,eta", [(0, 0.0, 0.0), (1, 0.03, 0.0), (2, 0.0, 0.05), (3, 0.02, 0.04)])
def test_rhs_equals_primitive_form(seed, nu, eta):
    n = 16
    X, rho, u, B, P = _primitive_trig_state(seed)
    prim = _evaluate([rho] + u + B + [P], X, n)
    rho_g, u_g, B_g, P_g = prim[0], prim[1:4], prim[4:7], prim[7]
    assert rho_g.min() > 0.5 and P_g.min() > 1.0
    U = I.conserved(rho_g, u_g, B_g, P_g, GAMMA)
    R = O.rhs(U, GAMMA, nu, eta)
    expect = _evaluate(_primitive_rhs(X, rho, u, B, P, GAMMA, nu, eta), X, n)
    for f in range(8):
        scale = max(np.abs(expect[f]).max(), 1e-300)
        err = np.abs(R[f] - expect[f]).max() / scale
        assert err < 1e-11, (I.FIELD_NAMES[f], err)


# --------------------------------------------------------------------------- #
# 2. linear waves                                                              #
# --------------------------------------------------------------------------- #

def _linear_operator(n, kvec, U0, nu, eta, eps=1e-6):
    """Complex 8x8 matrix M with d/dt a = M a for perturbations Re(a e^{ik.x})."""
    z, y, x = I.grid(n)
    ph = kvec[0] * x + kvec[1] * y + kvec[2] * z + 0 * x + 0 * y + 0 * z
    c, s = np.cos(ph), np.sin(ph)
    M = np.zeros((8, 8), complex)
    for f in range(8):
        Up = U0.copy()
        Um = U0.copy()
        Up[f] += eps * c
        Um[f] -= eps * c
        dR = (O.rhs(Up, GAMMA, nu, eta) - O.rhs(Um, GAMMA, nu, eta)) / (2 * eps)
        a = 2 * np.mean(dR * c, axis=(1, 2, 3))
        b = 2 * np.mean(dR * s, axis=(1, 2, 3))
        M[:, f] = a - 1j * b
    return M


def _uniform(n, rho0, B0, P0):
    U = np.zeros((8, n, n, n))
    U[0] = rho0
    U[4:7] = np.asarray(B0)[:, None, None, None]
    U[7] = P0 / (GAMMA - 1) + 0.5 * np.sum(np.asarray(B0) ** 2)
    return U


@pytest.mark.parametrize("theta", [0.3, 0.9, 1.3])
def test_ideal_wave_frequencies(theta):
    n, k = 8, 2.0
    rho0, P0, Bm = 1.3, 0.9, 1.1
    B0 = (Bm * np.cos(theta), Bm * np.sin(theta), 0.0)
    M = _linear_operator(n, (2, 0, 0), _uniform(n, rho0, B0, P0), 0.0, 0.0)
    lam = np.linalg.eigvals(M)
    cs2 = GAMMA * P0 / rho0
    va2 = Bm * Bm / rho0
    ct2 = np.cos(theta) ** 2
    disc = np.sqrt((cs2 + va2) ** 2 - 4 * cs2 * va2 * ct2)
    wf = k * np.sqrt(0.5 * (cs2 + va2 + disc))
    ws = k * np.sqrt(0.5 * (cs2 + va2 - disc))
    wa = k * np.sqrt(va2 * ct2)
    expect = np.sort([0, 0, ws, ws, wa, wa, wf, wf])
    assert np.max(np.abs(lam.real)) < 1e-6
    assert np.allclose(np.sort(np.abs(lam.imag)), expect, rtol=0, atol=1e-6)


def test_damped_parallel_waves():
    """k parallel to B0: the two Alfven pairs decay at (nu+eta)k^2/2 with
    frequency sqrt(k^2 v_A^2 - ((nu-eta)k^2/2)^2); the sound pair at (2/3)nu k^2
    (traceless strain); the k-parallel B component at eta k^2; entropy at 0."""
    n, k = 8, 2.0
    rho0, P0, Bm, nu, eta = 1.0, 0.8, 1.2, 0.05, 0.02
    M = _linear_operator(n, (0, 0, 2), _uniform(n, rho0, (0.0, 0.0, Bm), P0), nu, eta)
    lam = np.linalg.eigvals(M)
    cs2 = GAMMA * P0 / rho0
    ga = 0.5 * (nu + eta) * k * k
    wa = np.sqrt(k * k * Bm * Bm / rho0 - (0.5 * (nu - eta) * k * k) ** 2)
    gs = (2.0 / 3.0) * nu * k * k
    ws = np.sqrt(cs2 * k * k - gs * gs)
    expect = [0.0, -eta * k * k] + [complex(-ga, s * wa) for s in (1, -1, 1, -1)] + \
             [complex(-gs, s * ws) for s in (1, -1)]
    got = list(lam)
    for e in expect:
        i = int(np.argmin([abs(g - e) for g in got]))
        assert abs(got[i] - e) < 1e-6, (e, got)
        got.pop(i)


# --------------------------------------------------------------------------- #
# 3. exact nonlinear solution and special cases                                #
# --------------------------------------------------------------------------- #

def cp_alfven(n, t, axis=0, k=1, B0=1.0, b0=0.4, rho0=1.5, P0=0.7, nu=0.0):
    """Circularly polarised Alfven wave along `axis`; with nu = eta its amplitude
    decays as exp(-nu k^2 t) and the pressure rises by (gamma-1)(b0^2 - b^2)."""
    z, y, x = I.grid(n)
    coords = (x, y, z)
    a, b = (axis + 1) % 3, (axis + 2) % 3
    w = k * B0 / np.sqrt(rho0)
    amp = b0 * np.exp(-nu * k * k * t)
    ph = k * coords[axis] - w * t + 0 * x + 0 * y + 0 * z
    Bv = np.zeros((3, n, n, n))
    Bv[axis] = B0
    Bv[a] = amp * np.cos(ph)
    Bv[b] = amp * np.sin(ph)
    uv = np.zeros((3, n, n, n))
    uv[a] = -amp * np.cos(ph) / np.sqrt(rho0)
    uv[b] = -amp * np.sin(ph) / np.sqrt(rho0)
    rho = np.full((n, n, n), rho0)
    P = np.full((n, n, n), P0 + (GAMMA - 1) * (b0 * b0 - amp * amp))
    return I.conserved(rho, uv, Bv, P, GAMMA)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("nu", [0.0, 0.03])
def test_cp_alfven_exact_time_derivative(axis, nu):
    n, t, h = 16, 0.37, 1e-4
    U = cp_alfven(n, t, axis=axis, k=2, nu=nu)
    R = O.rhs(U, GAMMA, nu, nu)
    # time derivative of the exact solution by a 4th-order central difference
    dU = (-cp_alfven(n, t + 2 * h, axis, 2, nu=nu) + 8 * cp_alfven(n, t + h, axis, 2, nu=nu)
          - 8 * cp_alfven(n, t - h, axis, 2, nu=nu) + cp_alfven(n, t - 2 * h, axis, 2, nu=nu)) / (12 * h)
    scale = np.abs(dU).max()
    assert np.abs(R - dU).max() < 1e-9 * scale
    assert np.abs(R[0]).max() < 1e-12 and np.abs(R[7]).max() < 1e-11


def test_uniform_state_has_zero_rhs():
    n = 12
    U = _uniform(n, 1.7, (0.3, -0.2, 0.5), 2.0)
    U[1:4] = np.array([0.4, -0.1, 0.2])[:, None, None, None] * 1.7
    U[7] += 0.5 * 1.7 * (0.16 + 0.01 + 0.04)
    R = O.rhs(U, GAMMA, 0.01, 0.02)
    assert np.abs(R).max() < 1e-12


def test_mean_modes_of_conserved_rhs_vanish():
    c = I.config_small(16)
    R = O.rhs(c.U, c.gamma, c.nu, c.eta)
    for f in (0, 1, 2, 3, 7):
        assert abs(R[f].mean()) < 1e-13 * max(1.0, np.abs(R[f]).max())


def test_axis_permutation_equivariance():
    """Relabel axes x->y->z->x: fields move with the grid and vector components
    rotate; the RHS must transform the same way."""
    c = I.random_turbulence(12, nu=0.01, eta=0.02, seeds=(5, 6, 7))
    U = c.U

    def perm(V):
        # new(z', y', x') with x' = z, y' = x, z' = y: array axes (z, y, x) -> (y, x, z)
        W = np.transpose(V, (0, 2, 3, 1)).copy()
        out = W.copy()
        for base in (1, 4):  # vector components: new_x = old_z, new_y = old_x, new_z = old_y
            out[base + 0], out[base + 1], out[base + 2] = W[base + 2], W[base + 0], W[base + 1]
        return out

    R1 = perm(O.rhs(U, c.gamma, c.nu, c.eta))
    R2 = O.rhs(perm(U), c.gamma, c.nu, c.eta)
    assert np.abs(R1 - R2).max() < 1e-11 * np.abs(R1).max()
