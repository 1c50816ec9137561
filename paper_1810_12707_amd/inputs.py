"""Seeded synthetic initial conditions, shared by the HIP path and the oracle.

This module holds none of the method's arithmetic (no right-hand side, no
time stepping, no dealiasing of products): it only builds real-space FP64
fields of the shapes and statistics the paper's 3D runs use, from
counter-based random numbers, so that both sides of every parity check ingest
the same arrays.

Field order and layout: array (8, n, n, n), axes (field, z, y, x), fields
rho, m_x, m_y, m_z, B_x, B_y, B_z, E on the periodic box [0, 2*pi)^3 with
x_j = 2*pi*j/n.  Units are the normalised Heaviside-Lorentz ones of the
paper's Section V (magnetic pressure |B|^2/2), with an ideal-gas energy
E = P/(gamma-1) + rho|u|^2/2 + |B|^2/2.

Random numbers: SplitMix64 (Steele, Lea & Flood 2014), output i of seed s is
mix(s + (i+1) * 0x9E3779B97F4A7C15); two uniforms in (0, 1] feed one
Box-Muller pair.  Random vector fields are drawn directly as complex Gaussian
Fourier coefficients on the modes of the requested shells (white noise has
i.i.d. Gaussian coefficients, so this is white noise filtered to the shells),
shaped to an energy spectrum, made solenoidal by the projection
(I - k k^T / |k|^2), synthesised with an inverse real FFT and scaled to the
requested rms.  The draw for coefficient (component c, kz, ky, kx) uses the
counter index ((c*n + kz mod n)*n + ky mod n)*(n//2+1) + kx.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

FIELD_NAMES = ("rho", "m_x", "m_y", "m_z", "B_x", "B_y", "B_z", "E")


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Output number `counters` (0-based) of the SplitMix64 stream of `seed`."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1]: (top 53 bits + 1) * 2^-53."""
    z = splitmix64(seed, counters)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def normal_pair(seed: int, index: np.ndarray):
    """Box-Muller pair from uniforms number 2*index and 2*index+1."""
    index = np.asarray(index, dtype=np.uint64)
    u1 = uniform01(seed, np.uint64(2) * index)
    u2 = uniform01(seed, np.uint64(2) * index + np.uint64(1))
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def grid(n: int):
    """Coordinates (z, y, x) broadcastable to (n, n, n)."""
    x = 2.0 * np.pi * np.arange(n) / n
    return x[:, None, None], x[None, :, None], x[None, None, :]


def _irfftn(spec: np.ndarray, n: int) -> np.ndarray:
    try:
        import scipy.fft as sfft

        return sfft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2), workers=min(16, os.cpu_count() or 1))
    except ImportError:  # pragma: no cover
        return np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))


def shell_modes(n: int, k_lo: int, k_hi: int):
    """Integer modes (kz, ky, kx), kx >= 0, with shell index floor(|k| + 1/2) in
    [k_lo, k_hi] and 3|k_i| < n on every axis."""
    r = np.arange(-(k_hi + 1), k_hi + 2)
    kz, ky, kx = np.meshgrid(r, r, np.arange(0, k_hi + 2), indexing="ij")
    kz, ky, kx = kz.ravel(), ky.ravel(), kx.ravel()
    s = np.floor(np.sqrt(kx * kx + ky * ky + kz * kz) + 0.5)
    keep = (s >= k_lo) & (s <= k_hi) & (3 * np.abs(kx) < n) & (3 * np.abs(ky) < n) & (3 * np.abs(kz) < n)
    return kz[keep], ky[keep], kx[keep]


def shell_coefficients(n: int, seed: int, ncomp: int, k_lo: int, k_hi: int, slope: float | None = None,
                       solenoidal: bool = True, comp_offset: int = 0, spectrum=None):
    """The seeded Fourier coefficients of random_field (before its rms
    scaling): the modes (kz, ky, kx), kx >= 0, of shells [k_lo, k_hi] and an
    (ncomp, modes) complex array."""
    kz, ky, kx = shell_modes(n, k_lo, k_hi)
    nh = n // 2 + 1
    coef = np.zeros((ncomp, kz.size), dtype=np.complex128)
    for c in range(ncomp):
        idx = (((c + comp_offset) * n + (kz % n)) * n + (ky % n)) * nh + kx
        re, im = normal_pair(seed, idx.astype(np.uint64))
        coef[c] = re + 1j * im
    kk = np.sqrt((kx * kx + ky * ky + kz * kz).astype(np.float64))
    if slope is not None:
        coef *= kk ** ((slope - 2.0) / 2.0)
    if spectrum is not None:
        coef *= np.sqrt(spectrum(kk) / (kk * kk))
    if solenoidal:
        assert ncomp == 3
        kv = np.stack([kx, ky, kz]).astype(np.float64)  # component order x, y, z
        kdot = (kv * coef).sum(axis=0) / (kk * kk)
        coef = coef - kv * kdot
    return (kz, ky, kx), coef


def random_field(n: int, seed: int, ncomp: int, k_lo: int, k_hi: int, rms: float,
                 slope: float | None = None, solenoidal: bool = True, comp_offset: int = 0,
                 spectrum=None) -> np.ndarray:
    """Gaussian random field (ncomp, n, n, n) in shells [k_lo, k_hi].

    slope=alpha shapes the shell energy spectrum to E(k) ~ k^alpha (coefficient
    amplitude ~ |k|^((alpha-2)/2)); spectrum=E (a function of |k|) shapes it to
    E(|k|) (amplitude ~ (E(|k|) / |k|^2)^(1/2)); neither leaves it white.  rms
    is the target <|f|^2>^(1/2) over all components."""
    (kz, ky, kx), coef = shell_coefficients(n, seed, ncomp, k_lo, k_hi, slope, solenoidal, comp_offset, spectrum)
    nh = n // 2 + 1
    out = np.empty((ncomp, n, n, n), dtype=np.float64)
    for c in range(ncomp):
        spec = np.zeros((n, n, nh), dtype=np.complex128)
        spec[kz % n, ky % n, kx] = coef[c]
        out[c] = _irfftn(spec, n)
    cur = math.sqrt(float(np.mean(np.sum(out * out, axis=0))))
    if cur > 0:
        out *= rms / cur
    return out


def mode_planes(torch, n: int, modes, coef: np.ndarray, z0: int, z1: int, device=None):
    """Planes z0 <= z < z1 of the field random_field synthesises from `coef`
    (before its rms scaling), as an explicit sum over the few modes instead of
    a full-size inverse FFT: (ncomp, z1 - z0, n, n) FP64 torch tensor.  The
    inverse real FFT of a half spectrum holding coef_k at k = (kz, ky, kx),
    kx >= 0, is sum_k w_k Re(coef_k exp(i k.x)) / n^3 with w = 1 on the kx = 0
    plane (there the real transform keeps only the real part) and 2 elsewhere."""
    kz, ky, kx = modes
    f64 = torch.float64
    h = 2.0 * math.pi / n
    z = (torch.arange(z0, z1, dtype=f64, device=device) * h)[:, None, None]
    y = (torch.arange(n, dtype=f64, device=device) * h)[None, :, None]
    x = (torch.arange(n, dtype=f64, device=device) * h)[None, None, :]
    ncomp = coef.shape[0]
    out = torch.zeros((ncomp, z1 - z0, n, n), dtype=f64, device=device)
    n3 = float(n) ** 3
    for m in range(kz.size):
        th = (float(kz[m]) * z + float(ky[m]) * y) + float(kx[m]) * x
        c, s = torch.cos(th), torch.sin(th)
        w = (1.0 if kx[m] == 0 else 2.0) / n3
        for comp in range(ncomp):
            a = complex(coef[comp, m])
            out[comp].add_(c, alpha=w * a.real).add_(s, alpha=-w * a.imag)
    return out


def random_field_device(torch, n: int, seed: int, ncomp: int, k_lo: int, k_hi: int, rms: float, device=None,
                        chunk: int = 64, **kw):
    """random_field (up to rounding) built on `device`, plane chunk by plane
    chunk: (ncomp, n, n, n) FP64 tensor."""
    modes, coef = shell_coefficients(n, seed, ncomp, k_lo, k_hi, **kw)
    out = torch.empty((ncomp, n, n, n), dtype=torch.float64, device=device)
    ss = 0.0
    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        p = mode_planes(torch, n, modes, coef, z0, z1, device)
        out[:, z0:z1] = p
        ss += float(torch.sum(p * p))
    cur = math.sqrt(ss / float(n) ** 3)
    if cur > 0:
        out.mul_(rms / cur)
    return out


def abc_flow(n: int, A=1.0, B=1.0, C=1.0, k=1.0) -> np.ndarray:
    """Arnold-Beltrami-Childress flow of the paper's Section V-B."""
    z, y, x = grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = A * np.sin(k * z) + C * np.cos(k * y)
    u[1] = B * np.sin(k * x) + A * np.cos(k * z)
    u[2] = C * np.sin(k * y) + B * np.cos(k * x)
    return u


def conserved(rho, u, B, P, gamma) -> np.ndarray:
    """Primitive (rho, u, B, P) -> conserved (rho, m, B, E), (8, n, n, n)."""
    n = rho.shape[0]
    U = np.empty((8, n, n, n), dtype=np.float64)
    U[0] = rho
    U[1:4] = rho[None] * u
    U[4:7] = B
    U[7] = P / (gamma - 1.0) + 0.5 * rho * np.sum(u * u, axis=0) + 0.5 * np.sum(B * B, axis=0)
    return U


def cfl_dt(U: np.ndarray, gamma: float, courant: float = 0.1) -> float:
    """Time step courant * dx / max(max_i |u_i| + c_f), c_f^2 = (gamma P + |B|^2)/rho."""
    n = U.shape[1]
    rho = U[0]
    u = U[1:4] / rho
    B2 = np.sum(U[4:7] ** 2, axis=0)
    P = (gamma - 1.0) * (U[7] - 0.5 * rho * np.sum(u * u, axis=0) - 0.5 * B2)
    cf = np.sqrt((gamma * P + B2) / rho)
    smax = float(np.max(np.max(np.abs(u), axis=0) + cf))
    return courant * (2.0 * np.pi / n) / smax


@dataclass
class Case:
    """A synthetic workload: FP64 real fields plus the run parameters."""
    name: str
    U: np.ndarray
    gamma: float
    nu: float
    eta: float
    dt: float
    steps: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.U.shape[1]


def abc_dynamo(n: int = 32, nu: float = 1e-2, eta: float = 1e-2, dt: float | None = 1e-3,
               steps: int = 100, mach: float = 0.1, b_rms: float = 1e-3, seed: int = 0,
               gamma: float = 5.0 / 3.0, name: str = "abc") -> Case:
    """rho = 1, ABC velocity (U0 = 1), seeded white solenoidal B in shells 1-4
    with the given rms, uniform pressure from the sound speed U0/mach."""
    rho = np.ones((n, n, n))
    u = abc_flow(n)
    B = random_field(n, seed, 3, 1, 4, b_rms)
    cs = 1.0 / mach
    P = np.full((n, n, n), rho[0, 0, 0] * cs * cs / gamma)
    U = conserved(rho, u, B, P, gamma)
    if dt is None:
        dt = cfl_dt(U, gamma)
    return Case(name, U, gamma, nu, eta, dt, steps, {"mach": mach})


def random_turbulence(n: int = 256, nu: float = 2e-3, eta: float = 2e-3, steps: int = 1000,
                      mach: float = 0.3, b_rms: float = 0.1, seeds=(1, 2, 3),
                      gamma: float = 5.0 / 3.0, name: str = "turb") -> Case:
    """Solenoidal velocity with E(k) ~ k^-2 in shells 1-8 and rms 1; white
    solenoidal B in shells 1-4; rho = 1 + d with d in shells 1-8, max |d| =
    0.01; isentropic P = P0 rho^gamma with P0 = c_s^2/gamma, c_s = 1/mach."""
    u = random_field(n, seeds[0], 3, 1, 8, 1.0, slope=-2.0)
    B = random_field(n, seeds[1], 3, 1, 4, b_rms)
    d = random_field(n, seeds[2], 1, 1, 8, 1.0, solenoidal=False)[0]
    d *= 0.01 / float(np.max(np.abs(d)))
    rho = 1.0 + d
    cs = 1.0 / mach
    P = (cs * cs / gamma) * rho ** gamma
    U = conserved(rho, u, B, P, gamma)
    return Case(name, U, gamma, nu, eta, cfl_dt(U, gamma), steps, {"mach": mach})


def orszag_tang(n: int = 1024, nu: float = 5e-4, eta: float = 5e-4, steps: int = 50, seed: int = 4,
                amp: float = 1e-2, gamma: float = 5.0 / 3.0, name: str = "ot") -> Case:
    """3D Orszag-Tang-type start: u = (-sin y, sin x, 0), B = (-sin y, sin 2x, 0),
    plus seeded solenoidal shells 1-4 of rms `amp` in u and in B;
    rho = 25/9, P = 5/3."""
    z, y, x = grid(n)
    u = np.zeros((3, n, n, n))
    B = np.zeros((3, n, n, n))
    u[0] = -np.sin(y) + 0 * x + 0 * z
    u[1] = np.sin(x) + 0 * y + 0 * z
    B[0] = -np.sin(y) + 0 * x + 0 * z
    B[1] = np.sin(2 * x) + 0 * y + 0 * z
    u += random_field(n, seed, 3, 1, 4, amp)
    B += random_field(n, seed, 3, 1, 4, amp, comp_offset=3)
    rho = np.full((n, n, n), 25.0 / 9.0)
    P = np.full((n, n, n), 5.0 / 3.0)
    U = conserved(rho, u, B, P, gamma)
    return Case(name, U, gamma, nu, eta, cfl_dt(U, gamma), steps, {})


def orszag_tang_device(torch, n: int = 1024, device=None, dtype=None, nu: float = 5e-4, eta: float = 5e-4,
                       steps: int = 50, seed: int = 4, amp: float = 1e-2, gamma: float = 5.0 / 3.0,
                       name: str = "ot", chunk: int = 64) -> Case:
    """orszag_tang (up to rounding) built on `device` (no n^3 host array):
    Case whose U is an (8, n, n, n) torch tensor of `dtype` (FP32 unless
    given) on that device."""
    f64 = torch.float64
    dtype = dtype or torch.float32
    h = 2.0 * math.pi / n
    u = random_field_device(torch, n, seed, 3, 1, 4, amp, device, chunk)
    B = random_field_device(torch, n, seed, 3, 1, 4, amp, device, chunk, comp_offset=3)
    x = torch.arange(n, dtype=f64, device=device) * h
    u[0] -= torch.sin(x)[None, :, None]
    u[1] += torch.sin(x)[None, None, :]
    B[0] -= torch.sin(x)[None, :, None]
    B[1] += torch.sin(2.0 * x)[None, None, :]
    rho, P = 25.0 / 9.0, 5.0 / 3.0
    U = torch.empty((8, n, n, n), dtype=dtype, device=device)
    smax = 0.0
    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        uc, Bc = u[:, z0:z1], B[:, z0:z1]
        u2, B2 = torch.sum(uc * uc, dim=0), torch.sum(Bc * Bc, dim=0)
        U[0, z0:z1] = rho
        U[1:4, z0:z1] = (rho * uc).to(dtype)
        U[4:7, z0:z1] = Bc.to(dtype)
        U[7, z0:z1] = (P / (gamma - 1.0) + 0.5 * rho * u2 + 0.5 * B2).to(dtype)
        cf = torch.sqrt((gamma * P + B2) / rho)
        smax = max(smax, float(torch.max(torch.amax(torch.abs(uc), dim=0) + cf)))
    del u, B
    dt = 0.1 * h / smax
    return Case(name, U, gamma, nu, eta, dt, steps, {})


def compressive_state(n: int, seed: int, gamma: float = 5.0 / 3.0) -> np.ndarray:
    """A test start whose right-hand side is well conditioned in FP32: a
    general (half compressive) velocity of rms 0.5 in shells 1-4, solenoidal
    B of rms 0.3, rho = 1 + 20% and P = 0.6 + 0.1 rms noise in shells 1-4 (a
    modest background pressure, so -div F^E is not a small difference of
    large terms, and div m is not that of a nearly solenoidal flow)."""
    u = random_field(n, seed, 3, 1, 4, 0.5, solenoidal=False)
    B = random_field(n, seed + 1, 3, 1, 4, 0.3)
    d = random_field(n, seed + 2, 1, 1, 4, 1.0, solenoidal=False)[0]
    rho = 1.0 + 0.2 * d / float(np.max(np.abs(d)))
    P = 0.6 + random_field(n, seed + 3, 1, 1, 4, 0.1, solenoidal=False)[0]
    return conserved(rho, u, B, P, gamma)


@dataclass
class TrigState:
    """Primitive fields that are trigonometric polynomials with wavevectors in
    {-1, 0, 1}^3 (degree <= 1 per axis): each field is a constant plus a few
    terms amp * cos(k.x + phase).  B_i depends only on the two coordinates
    other than x_i, so div B = 0 exactly."""
    terms: dict  # name -> (constant, [(amp, (kx, ky, kz), phase), ...])

    def evaluate(self, name: str, z, y, x, xp=np):
        c0, ts = self.terms[name]
        out = c0 + 0.0 * (x + y + z)
        for amp, (kx, ky, kz), ph in ts:
            out = out + amp * xp.cos(kx * x + ky * y + kz * z + ph)
        return out

    def conserved(self, z, y, x, gamma: float, xp=np):
        """rho, m = rho u, B, E = P/(gamma-1) + rho|u|^2/2 + |B|^2/2 at the
        given coordinates (numpy or torch arrays), stacked (8, ...)."""
        rho = self.evaluate("rho", z, y, x, xp)
        u = [self.evaluate(f"u{i}", z, y, x, xp) for i in range(3)]
        B = [self.evaluate(f"B{i}", z, y, x, xp) for i in range(3)]
        P = self.evaluate("P", z, y, x, xp)
        E = P / (gamma - 1.0) + 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + \
            0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2])
        return xp.stack([rho, rho * u[0], rho * u[1], rho * u[2], B[0], B[1], B[2], E])


def trig_state(seed: int, rho_amp: float = 0.15, u_amp: float = 0.4, b_amp: float = 0.4,
               p_amp: float = 0.1, p0: float = 1.0) -> TrigState:
    """Random TrigState (numpy's seeded generator): three terms per field.
    With m = rho u and E as in TrigState.conserved every flux of Eqs.
    MHD1-MHD4 is a trigonometric polynomial of degree <= 4 per axis, so the
    right-hand side is the same polynomial on every grid with n >= 13."""
    rng = np.random.default_rng(seed)

    def terms(scale, kset=None):
        out = []
        for _ in range(3):
            k = [int(v) for v in rng.integers(-1, 2, size=3)]
            if kset is not None:
                k = [k[j] if kset[j] else 0 for j in range(3)]
            out.append((float(rng.uniform(-1, 1) * scale), tuple(k), float(rng.uniform(0, 2 * np.pi))))
        return out

    t = {"rho": (1.0, terms(rho_amp / 3)), "P": (p0, terms(p_amp / 3))}
    for i in range(3):
        t[f"u{i}"] = (float(rng.uniform(-0.2, 0.2)), terms(u_amp / 3))
        mask = [j != i for j in range(3)]  # (x, y, z): B_i independent of x_i
        t[f"B{i}"] = (float(rng.uniform(-0.3, 0.3)), terms(b_amp / 3, mask))
    return TrigState(t)


def decaying_turbulence(n: int = 64, k0: float = 4.0, mach: float = 0.1, nu: float = 2e-3,
                        seed: int = 8, gamma: float = 5.0 / 3.0, name: str = "decay") -> Case:
    """The hydrodynamic decaying-turbulence start of Section V-A: rho = 1,
    solenoidal u with E(k) = A k^4 exp(-2 k^2 / k0^2) over every retained
    shell, rms 1 (<|u|^2>^(1/2) = U0 = 1), uniform P from the Mach number
    (c_s = U0 / M), B = 0, nu = eta; dt from the CFL condition."""
    K = (n - 1) // 3
    u = random_field(n, seed, 3, 1, K, 1.0, spectrum=lambda k: k ** 4 * np.exp(-2.0 * k * k / (k0 * k0)))
    rho = np.ones((n, n, n))
    cs = 1.0 / mach
    P = np.full((n, n, n), cs * cs / gamma)
    U = conserved(rho, u, np.zeros((3, n, n, n)), P, gamma)
    return Case(name, U, gamma, nu, nu, cfl_dt(U, gamma), 1000, {"mach": mach, "k0": k0})


# The workloads of the paper's 3D MHD runs as concrete synthetic inputs.
def config_small(n: int = 32) -> Case:
    """32^3 ABC-flow start, B rms 1e-3 in shells 1-4 (seed 0), Mach 0.1,
    nu = eta = 1e-2, dt = 1e-3, 100 AB2 steps."""
    return abc_dynamo(n, 1e-2, 1e-2, 1e-3, 100, name=f"abc{n}")


def config_turb256(n: int = 256) -> Case:
    """256^3 random-phase turbulence, Mach 0.3, nu = eta = 2e-3, 1000 steps."""
    return random_turbulence(n, name=f"turb{n}")


def config_dynamo512(n: int = 512) -> Case:
    """512^3 ABC dynamo start, nu = eta = 1e-3, dt = CFL(0.1), 200 steps."""
    return abc_dynamo(n, 1e-3, 1e-3, None, 200, name=f"abc{n}")


def config_ot1024(n: int = 1024) -> Case:
    """1024^3 Orszag-Tang-type start, nu = eta = 5e-4, 50 steps."""
    return orszag_tang(n, name=f"ot{n}")


# Stream of the ensemble's per-run diffusivities (independent of the field seeds).
ENSEMBLE_PARAM_SEED = 0x5EED_0E15


def ensemble_member(i: int, n: int, steps: int = 500, mach: float = 0.3, b_rms: float = 0.1) -> Case:
    """Run i of the batched ensemble: random-phase turbulence (as
    random_turbulence) from seed i, with nu = eta = 10^(-3 + v), v uniform in
    (0, 1] (log-uniform in [1e-3, 1e-2]), dt from the CFL condition."""
    v = float(uniform01(ENSEMBLE_PARAM_SEED, np.array([i]))[0])
    nu = 10.0 ** (-3.0 + v)
    return random_turbulence(n, nu=nu, eta=nu, steps=steps, mach=mach, b_rms=b_rms,
                             seeds=(i, 1000 + i, 2000 + i), name=f"ens{i}_n{n}")


def config_ensemble(count: int = 64, sizes=(32, 64, 96, 128), steps: int = 500) -> list:
    """The batched ensemble: `count` runs, sizes in equal consecutive blocks
    (16 each of 32^3, 64^3, 96^3, 128^3 by default: 52.4 M points), seeds
    0..count-1, FP32, 500 steps."""
    per = max(1, count // len(sizes))
    return [ensemble_member(i, sizes[min(i // per, len(sizes) - 1)], steps) for i in range(count)]
