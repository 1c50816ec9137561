"""Parity at the benchmark sizes (256^3, 512^3), in the launch configuration
bench.py times, on outputs that can be checked one by one or through
properties that hold at any size.

* Transforms: sampled coefficients of mhd_fft3d on a random field against the
  DFT sum itself (FP64, separable direct sums; no FFT involved).
* RHS: a state with rho = 1 and only |k_i| <= 2 modes in m, B, E.  Every flux
  is then a polynomial of degree <= 3 in the state, so the exact RHS has modes
  |k_i| <= 6 only and the discrete RHS is the same trigonometric polynomial at
  every n >= 32 (no truncation by the 2/3 mask, no aliasing).  The oracle's
  RHS at 32^3 gives its Fourier coefficients, which are summed directly at
  sampled points of the large grid.
* Steps: ten steps of the benchmark workloads keep the means of rho, m and E
  (their k = 0 right-hand sides vanish identically) and div B = 0 up to
  rounding.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_12707_amd import inputs as I
from tests.gpu_helpers import band, compact_from_flat, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def solver(n, prec, **kw):
    from paper_1810_12707_amd.mhd import Solver

    return Solver(n, precision=prec, **kw)


def sampled_dft(f, ks):
    """f^(k) = sum_x f(x) exp(-i k.x) for the wavenumber triples ks (FP64)."""
    n = f.shape[0]
    xs = np.arange(n)
    kx_set = sorted({k[0] for k in ks})
    Ex = np.exp(-2j * np.pi * np.outer(xs, kx_set) / n)            # [x][j]
    A = (f.reshape(n * n, n).astype(np.float64) @ Ex).reshape(n, n, len(kx_set))  # [z][y][j]
    out = []
    for kx, ky, kz in ks:
        j = kx_set.index(kx)
        ey = np.exp(-2j * np.pi * ky * xs / n)
        ez = np.exp(-2j * np.pi * kz * xs / n)
        out.append(ez @ (A[:, :, j] @ ey))
    return np.array(out)


@pytest.mark.parametrize("n,prec", [(256, "fp32"), (512, "fp32"), (512, "mixed"), (1024, "fp32")])
def test_fft_sampled_coefficients(n, prec):
    """Mixed: the BF16 split keeps ~16 bits per product, so its bar is the
    mixed transform bar (2e-4 relative L2) with the max-over-samples margin."""
    log(f"[fullsize fft] n={n} prec={prec}")
    rng = np.random.default_rng(7 + n)
    f = rng.standard_normal((n, n, n), dtype=np.float32)
    S = solver(n, prec)
    spec = S.fft_forward(torch.from_numpy(f).to("cuda:0"))
    torch.cuda.synchronize()
    K, nb, _ = band(n)
    # 48 random retained modes (kx from 6 values) plus the corners of the band
    kx_pool = [0, K] + [int(v) for v in rng.integers(1, K, size=4)]
    ks = [(int(rng.choice(kx_pool)), int(rng.integers(-K, K + 1)), int(rng.integers(-K, K + 1))) for _ in range(48)]
    ks += [(0, 0, 0), (K, K, K), (K, -K, -K), (0, K, -K), (K, 0, 0)]
    got_all = compact_from_flat(spec.cpu().numpy(), n)  # [kz][ky][kx] band order
    got = np.array([got_all[kz % nb, ky % nb, kx] for kx, ky, kz in ks])
    ref = sampled_dft(f, ks)
    scale = n ** 1.5  # rms of a coefficient of unit white noise
    err = np.max(np.abs(got - ref)) / scale
    log(f"  max |error| / n^1.5 = {err:.3e}")
    assert err <= (1e-5 if prec == "fp32" else 2e-3)
    S.close()


def lowmode_state(n0=32, seed=11):
    """rho = 1; m, B (solenoidal), E = 3 + e with only |k_i| <= 2 modes, at n0^3."""
    def lowmodes(ncomp, rms, s, solenoidal):
        return I.random_field(n0, s, ncomp, 1, 2, rms, solenoidal=solenoidal)

    m = lowmodes(3, 0.3, seed, False)
    B = lowmodes(3, 0.3, seed + 1, True)
    e = lowmodes(1, 0.1, seed + 2, False)[0]
    # shells 1-2 hold |k| <= 2.5; keep only |k_i| <= 2 per axis (cube) explicitly
    def cube(a):
        F = np.fft.fftn(a, axes=(-3, -2, -1))
        k = np.fft.fftfreq(n0, 1.0 / n0)
        kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
        F[..., (np.abs(kx) > 2) | (np.abs(ky) > 2) | (np.abs(kz) > 2)] = 0
        return np.real(np.fft.ifftn(F, axes=(-3, -2, -1)))
    U = np.empty((8, n0, n0, n0))
    U[0] = 1.0
    U[1:4] = cube(m)
    U[4:7] = cube(B)
    U[7] = 3.0 + cube(e[None])[0]
    return U


def upsample_field(a, n, kmax=2):
    """The trigonometric polynomial of one n0^3 field with modes |k_i| <= kmax,
    sampled on an n^3 grid (zero-padded inverse real FFT, FP64)."""
    import scipy.fft as sf

    n0 = a.shape[-1]
    F = sf.rfftn(a) / n0 ** 3
    G = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    ks = np.r_[0:kmax + 1, -kmax:0]
    G[np.ix_(ks % n, ks % n, np.arange(kmax + 1))] = F[np.ix_(ks % n0, ks % n0, np.arange(kmax + 1))]
    return sf.irfftn(G, s=(n, n, n), workers=8) * n ** 3


def upsample_field_gpu(a, n, kmax=2):
    """As upsample_field, evaluated on the GPU in FP64 by separable sums over
    the few modes (x, then y, then z): returns an n^3 float64 CUDA tensor."""
    n0 = a.shape[-1]
    F = np.fft.fftn(a) / n0 ** 3                     # [kz][ky][kx]
    ks = np.r_[-kmax:kmax + 1]
    C = torch.from_numpy(np.ascontiguousarray(F[np.ix_(ks % n0, ks % n0, ks % n0)])).to("cuda:0")
    x = torch.arange(n, device="cuda:0", dtype=torch.float64) * (2 * np.pi / n)
    kk = torch.from_numpy(ks.astype(np.float64)).to("cuda:0")
    E = torch.exp(1j * torch.outer(kk, x))           # [k][x] complex128
    m = len(ks)
    A = (C.reshape(m * m, m) @ E).reshape(m, m, n)  # [kz][ky][x]
    A = (A.permute(0, 2, 1).reshape(m * n, m) @ E).reshape(m, n, n).permute(0, 2, 1)  # [kz][y][x]
    A = A.reshape(m, n * n)
    out = (E.real.transpose(0, 1).contiguous() @ A.real.contiguous()
           - E.imag.transpose(0, 1).contiguous() @ A.imag.contiguous())                  # [z][y x]
    return out.reshape(n, n, n)


def eval_points(coef, kvec, pts, n):
    """sum_k coef[k] exp(i k.x) at grid points pts (z, y, x indices) of the n grid."""
    x = 2 * np.pi * pts[:, ::-1] / n            # (x, y, z)
    ph = np.exp(1j * (x @ kvec.T))              # [points][modes]
    return np.real(ph @ coef.T).T               # [fields][points]


def low_mode_coefficients(R, kmax):
    """(1/n^3) sum_x R_f(x) exp(-i k.x) for |k_i| <= kmax of real fields R
    ([F][n][n][n], on the GPU), as [F][kz][ky][kx] with k = -kmax..kmax
    (separable direct sums in FP64)."""
    F_, n = R.shape[0], R.shape[-1]
    m = 2 * kmax + 1
    k = torch.arange(-kmax, kmax + 1, device=R.device, dtype=torch.float64)
    x = torch.arange(n, device=R.device, dtype=torch.float64)
    E = torch.exp(-2j * np.pi * torch.outer(x, k) / n)                       # [x][k]
    out = torch.empty((F_, m, m, m), dtype=torch.complex128, device=R.device)
    for f in range(F_):
        A = R[f].double().reshape(n * n, n).to(torch.complex128) @ E          # [z y][kx]
        A = A.reshape(n, n, m).permute(0, 2, 1).reshape(n * m, n) @ E          # [z kx][ky]
        A = A.reshape(n, m * m).transpose(0, 1).contiguous() @ E               # [kx ky][kz]
        out[f] = A.reshape(m, m, m).permute(2, 1, 0) / n ** 3                  # [kz][ky][kx]
    return out


@pytest.mark.parametrize("n,prec", [(256, "fp32"), (512, "fp32"), (256, "fp64"), (512, "fp64"), (256, "mixed"),
                                    (512, "mixed"), (1024, "fp32"), (1024, "mixed"),
                                    # radix-3 plans (8,8,3), (8,4,4,3), (8,8,4,3) under both row layouts
                                    (192, "fp32"), (384, "fp32"), (768, "fp32")])
def test_rhs_exact_lowmode_state(n, prec):
    """FP64: pointwise at sampled grid points.  FP32: the rounding of P ~ 2 to
    FP32 is white noise over every mode up to K, and the divergence multiplies
    mode k by |k| <= sqrt(3) K, so pointwise FP32 errors grow ~ eps |P| K / |R|
    (~3e-5 at 256^3).  The operator itself is checked on the modes |k_i| <= 6
    that hold the exact answer (noise there is ~(13/(2K+1))^1.5 smaller), and
    the energy left outside them is bounded by that rounding estimate."""
    log(f"[fullsize rhs] n={n} prec={prec}")
    gamma, nu, eta = 5.0 / 3.0, 2e-3, 3e-3
    n0 = 32
    U0 = lowmode_state(n0)
    R0 = O.rhs(U0, gamma, nu, eta)                       # oracle, FP64, 32^3
    F = np.fft.fftn(R0, axes=(-3, -2, -1)) / n0 ** 3
    k = np.fft.fftfreq(n0, 1.0 / n0).astype(int)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    keep = (np.abs(kx) <= 6) & (np.abs(ky) <= 6) & (np.abs(kz) <= 6)
    # the exact RHS lives on |k_i| <= 6: nothing else may be present
    assert np.max(np.abs(F[:, ~keep])) <= 1e-12 * np.max(np.abs(F))
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    Un = torch.empty((8, n, n, n), dtype=dt_, device="cuda:0")
    for f in range(8):
        Un[f] = upsample_field_gpu(U0[f], n).to(dt_)
    S = solver(n, prec, gamma=gamma, nu=nu, eta=eta)
    out = S.rhs(Un)
    del Un
    if prec == "fp64":
        kvec = np.stack([kx[keep], ky[keep], kz[keep]], axis=1).astype(np.float64)
        coef = F[:, keep]
        rng = np.random.default_rng(5)
        pts = rng.integers(0, n, size=(4096, 3))
        pt = torch.from_numpy(pts).to("cuda:0")
        got = out[:, pt[:, 0], pt[:, 1], pt[:, 2]].double().cpu().numpy()
        ref = eval_points(coef, kvec, pts.astype(np.float64), n)
        for f in range(8):
            e = np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])
            log(f"  field {I.FIELD_NAMES[f]}: rel L2 at sampled points {e:.3e}")
            assert e <= 1e-11, (f, e)
    else:
        idx = np.r_[-6:7] % n0
        exact = F[:, idx[:, None, None], idx[None, :, None], idx[None, None, :]]    # [f][kz][ky][kx]
        got = low_mode_coefficients(out, 6).cpu().numpy()
        K = (n - 1) // 3
        noise = 1.2e-7 * 3.0 * np.sqrt(3.0) * K        # eps * |P|-scale * max |k|, absolute
        low_tol = 1e-5
        if prec == "mixed":  # BF16 split: ~2^8 x the FP32 rounding per product, the mixed bound 1e-3
            noise *= 256.0
            low_tol = 1e-3
        for f in range(8):
            e = np.linalg.norm(got[f] - exact[f]) / np.linalg.norm(exact[f])
            tot = float(torch.linalg.vector_norm(out[f].double())) ** 2 / n ** 3      # <R^2>
            low = float(np.sum(np.abs(got[f]) ** 2))                                  # Parseval, |k_i| <= 6
            rest = np.sqrt(max(tot - low, 0.0))
            log(f"  field {I.FIELD_NAMES[f]}: low modes rel {e:.3e}; rms outside {rest:.3e} "
                f"(bound {noise:.1e}, rms R {np.sqrt(low):.3e})")
            assert e <= low_tol, (f, e)
            assert rest <= noise, (f, rest, noise)
    S.close()


@pytest.mark.parametrize("case_name,n,prec", [("turb", 256, "fp32"), ("abc", 512, "fp32"), ("turb", 256, "mixed"),
                                              ("abc", 512, "mixed")])
def test_ten_steps_conserve(case_name, n, prec):
    """The k = 0 right-hand sides of rho, m and E vanish identically, whatever
    the transforms' rounding, so the means hold at FP32 rounding on both
    paths.  div B of the state sits at the transforms' own error level (the
    forward transform of the initial fields already puts it there: ~1e-6 of
    the current in FP32, 4e-5 to 7e-5 on the mixed path, under its transform
    bound 2e-4) and the curl-form induction update must not make it grow."""
    log(f"[fullsize steps] {case_name} n={n} prec={prec}")
    c = I.config_turb256(n) if case_name == "turb" else I.config_dynamo512(n)
    S = solver(n, prec, gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt)
    S.set_state(torch.from_numpy(c.U).to("cuda:0"))
    rc0, d0 = S.diagnostics()
    S.step(10)
    rc1, d1 = S.diagnostics()
    log(f"  mass {d0['mass']:.9f} -> {d1['mass']:.9f}; E {d0['e_tot']:.7f} -> {d1['e_tot']:.7f}; "
        f"divB rel {d0['divb_rel']:.2e} -> {d1['divb_rel']:.2e}")
    assert rc0 == 0 and rc1 == 0
    assert abs(d1["mass"] - d0["mass"]) <= 1e-6 * abs(d0["mass"])
    assert abs(d1["e_tot"] - d0["e_tot"]) <= 1e-6 * abs(d0["e_tot"])
    scale = np.sqrt(2 * d0["e_kin"] * d0["mass"])  # ~ rms |m|
    for i in range(3):
        assert abs(d1["mom"][i] - d0["mom"][i]) <= 1e-6 * scale
    assert d1["divb_rel"] <= (1e-5 if prec == "fp32" else 2e-4)
    assert d1["divb_rel"] <= 1.5 * d0["divb_rel"] + 1e-7
    S.close()
