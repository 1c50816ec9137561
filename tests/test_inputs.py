"""The seeded input generators shared by the oracle and the HIP path (CPU
only): the counter-based generator against its published definition, and the
stated properties of each recipe (band, shells, rms, divergence, spectra)."""
import numpy as np
import pytest

from paper_1810_12707_amd import inputs as I

MASK = (1 << 64) - 1


def splitmix64_ref(seed, count):
    """SplitMix64 as published (Steele, Lea and Flood 2014; Vigna's reference
    code): add the golden gamma to the state, then mix with two xor-shift
    multiplies; written here as a scalar state machine."""
    out, s = [], seed & MASK
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_matches_its_definition():
    # first output of the stream of seed 0, as listed with the reference code
    assert int(I.splitmix64(0, np.array([0]))[0]) == 0xE220A8397B1DCDAF
    for seed in (0, 1, 12345, 2**63 + 7):
        got = I.splitmix64(seed, np.arange(20, dtype=np.uint64))
        assert [int(v) for v in got] == splitmix64_ref(seed, 20)
    # counter-based: any subset of counters gives the same numbers
    idx = np.array([19, 3, 7], dtype=np.uint64)
    assert [int(v) for v in I.splitmix64(5, idx)] == [splitmix64_ref(5, 20)[i] for i in (19, 3, 7)]


def test_uniform_and_normal_ranges():
    u = I.uniform01(3, np.arange(200000, dtype=np.uint64))
    assert u.min() > 0.0 and u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    a, b = I.normal_pair(4, np.arange(100000, dtype=np.uint64))
    z = np.concatenate([a, b])
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1.0) < 1e-2


def spectrum(f):
    return np.fft.fftn(f, axes=(-3, -2, -1))


def kgrid(n):
    k = np.fft.fftfreq(n, 1.0 / n)
    return k[:, None, None], k[None, :, None], k[None, None, :]  # kz, ky, kx


@pytest.mark.parametrize("n", [16, 24])
def test_random_field_properties(n):
    f = I.random_field(n, 7, 3, 1, 4, 0.5)
    assert np.array_equal(f, I.random_field(n, 7, 3, 1, 4, 0.5))  # seeded
    assert not np.array_equal(f, I.random_field(n, 8, 3, 1, 4, 0.5))
    assert abs(np.sqrt(np.mean(np.sum(f * f, axis=0))) - 0.5) < 1e-12
    F = spectrum(f)
    kz, ky, kx = kgrid(n)
    # solenoidal: k . F = 0 mode by mode
    div = kx * F[0] + ky * F[1] + kz * F[2]
    assert np.abs(div).max() <= 1e-12 * np.abs(F).max() * n
    # support: shells 1..4 and inside the 2/3 band on every axis
    shell = np.floor(np.sqrt(kx * kx + ky * ky + kz * kz) + 0.5)
    inside = (shell >= 1) & (shell <= 4) & (3 * np.abs(kx) < n) & (3 * np.abs(ky) < n) & (3 * np.abs(kz) < n)
    power = np.sum(np.abs(F) ** 2, axis=0)
    assert power[~inside].sum() <= 1e-24 * power.sum()


def test_spectral_slope():
    n = 32
    u = I.random_field(n, 11, 3, 1, 8, 1.0, slope=-2.0)
    F = spectrum(u)
    kz, ky, kx = kgrid(n)
    shell = np.floor(np.sqrt(kx * kx + ky * ky + kz * kz) + 0.5)
    power = np.sum(np.abs(F) ** 2, axis=0)
    E = np.array([power[shell == s].sum() for s in range(1, 9)])
    # E(k) ~ k^-2: the fitted log-log slope over shells 1-8
    slope = np.polyfit(np.log(np.arange(1, 9)), np.log(E), 1)[0]
    assert abs(slope + 2.0) < 0.35, slope


def test_abc_flow_is_beltrami():
    n = 16
    u = I.abc_flow(n, A=1.0, B=0.7, C=0.4)
    F = spectrum(u)
    kz, ky, kx = kgrid(n)
    curl = np.stack([1j * (ky * F[2] - kz * F[1]), 1j * (kz * F[0] - kx * F[2]), 1j * (kx * F[1] - ky * F[0])])
    assert np.abs(curl - F).max() <= 1e-12 * np.abs(F).max()  # curl u = k u with k = 1
    assert np.abs(kx * F[0] + ky * F[1] + kz * F[2]).max() <= 1e-12 * np.abs(F).max()


def test_turbulence_recipe():
    c = I.random_turbulence(24, b_rms=0.3)
    rho, m, B = c.U[0], c.U[1:4], c.U[4:7]
    u = m / rho
    d = rho - 1.0
    assert abs(np.abs(d).max() - 0.01) < 1e-12
    assert abs(np.sqrt(np.mean(np.sum(u * u, axis=0))) - 1.0) < 1e-12
    assert abs(np.sqrt(np.mean(np.sum(B * B, axis=0))) - 0.3) < 1e-12
    P = (c.gamma - 1.0) * (c.U[7] - 0.5 * np.sum(m * u, axis=0) - 0.5 * np.sum(B * B, axis=0))
    P0 = (1.0 / 0.3) ** 2 / c.gamma  # isentropic, sound speed 1 / mach at rho = 1
    assert np.allclose(P, P0 * rho ** c.gamma, rtol=1e-12)
    assert c.dt > 0 and np.isfinite(c.dt)


@pytest.mark.parametrize("n", [16, 24])
def test_device_builders_equal_the_host_recipes(n):
    """The mode-by-mode device builders (used where an n^3 host array and a
    full-size inverse FFT would take minutes, 1024^3) synthesise the same
    fields as the host recipes: random_field with and without the solenoidal
    projection, and the Orszag-Tang start with its CFL step (run here on the
    CPU through torch)."""
    torch = pytest.importorskip("torch")
    a = I.random_field(n, 7, 3, 1, 4, 0.3, comp_offset=3)
    b = I.random_field_device(torch, n, 7, 3, 1, 4, 0.3, chunk=5, comp_offset=3).numpy()
    assert np.abs(a - b).max() <= 1e-13
    a = I.random_field(n, 9, 1, 1, 4, 1.0, solenoidal=False)
    b = I.random_field_device(torch, n, 9, 1, 1, 4, 1.0, chunk=n, solenoidal=False).numpy()
    assert np.abs(a - b).max() <= 1e-13
    c = I.orszag_tang(n, name="ot")
    d = I.orszag_tang_device(torch, n, dtype=torch.float64, chunk=7)
    assert np.abs(c.U - d.U.numpy()).max() <= 1e-13 * np.abs(c.U).max()
    assert abs(c.dt - d.dt) <= 1e-14 * c.dt
