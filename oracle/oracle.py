"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports it.

Arrays are numpy float64 / complex128, C-contiguous; a real field set is
shaped (8, n, n, n) with axes (field, z, y, x) and field order
rho, m_x, m_y, m_z, B_x, B_y, B_z, E.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DIAG_NAMES = (
    "mass", "mom_x", "mom_y", "mom_z", "e_kin", "e_mag", "e_int", "e_tot",
    "h_cross", "h_mag", "divb_rms", "divb_max", "divb_rel", "dt_cfl", "c_s",
    "v_a", "mach_s", "mach_a", "nonfinite", "j_rms",
)


# time integrators and options (oracle.h)
SCHEMES = {"ab2": 0, "rk4": 1, "pc": 2}
VISC_LAPLACIAN, KINEMATIC = 1, 2


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("options", ctypes.c_int32),
        ("force", ctypes.c_double),
    ]


def build() -> str:
    """Compile liboracle.so in place (gcc, OpenMP)."""
    subprocess.run(["make", "-s", "-C", _HERE, "-B", "liboracle.so"], check=True)
    return _LIBPATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        L = ctypes.CDLL(_LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_fft1d.argtypes = [ctypes.c_int32, dp, dp, ctypes.c_int32]
        L.orc_fft3d.argtypes = [ctypes.c_int32, dp, ctypes.c_int32]
        L.orc_project.argtypes = [ctypes.c_int32, dp]
        L.orc_rhs.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.orc_run.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int32]
        L.orc_diag.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.orc_neumaier_sum.argtypes = [dp, ctypes.c_int64]
        L.orc_neumaier_sum.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int32
        L.orc_set_num_threads.argtypes = [ctypes.c_int32]
        L.orc_spectra.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int32, dp, dp, dp]
        L.orc_spectra.restype = ctypes.c_int
        L.orc_cic.argtypes = [ctypes.c_int32, dp, ctypes.c_int32, dp, ctypes.c_int64, dp]
        L.orc_cic.restype = ctypes.c_int
        L.orc_tracer_push.argtypes = [ctypes.c_int32, dp, dp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32]
        L.orc_tracer_push.restype = ctypes.c_int
        L.orc_set_num_threads.restype = None
        for name in ("orc_fft1d", "orc_fft3d", "orc_project", "orc_rhs", "orc_run", "orc_diag"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _params(n, gamma=5.0 / 3.0, nu=0.0, eta=0.0, dt=0.0, cfl=0.1, scheme="ab2", options=0,
            force=0.0) -> _Params:
    return _Params(int(n), float(gamma), float(nu), float(eta), float(dt), float(cfl), SCHEMES[scheme],
                   int(options), float(force))


def fft1d(x, sign: int = -1) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    _check(lib().orc_fft1d(x.size, _ptr(x.view(np.float64)), _ptr(out.view(np.float64)), sign), "fft1d")
    return out


def fft3d(a, sign: int = -1) -> np.ndarray:
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    n = a.shape[0]
    assert a.shape == (n, n, n)
    _check(lib().orc_fft3d(n, _ptr(a.view(np.float64)), sign), "fft3d")
    return a


def project(f) -> np.ndarray:
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_project(f.shape[0], _ptr(f)), "project")
    return f


def _fields(U) -> np.ndarray:
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    assert U.ndim == 4 and U.shape[0] == 8 and U.shape[1] == U.shape[2] == U.shape[3]
    return U


def rhs(U, gamma=5.0 / 3.0, nu=0.0, eta=0.0, options=0, force=0.0) -> np.ndarray:
    """options: VISC_LAPLACIAN | KINEMATIC; force: ABC body-force amplitude."""
    U = _fields(U)
    R = np.empty_like(U)
    p = _params(U.shape[1], gamma, nu, eta, options=options, force=force)
    _check(lib().orc_rhs(ctypes.byref(p), _ptr(U), _ptr(R)), "rhs")
    return R


def run(U, nsteps: int, dt: float, gamma=5.0 / 3.0, nu=0.0, eta=0.0, scheme="ab2", options=0,
        force=0.0) -> np.ndarray:
    """scheme: "ab2", "rk4" or "pc" (AB2 predictor, trapezoidal corrector)."""
    U = _fields(U)
    p = _params(U.shape[1], gamma, nu, eta, dt, scheme=scheme, options=options, force=force)
    _check(lib().orc_run(ctypes.byref(p), _ptr(U), int(nsteps)), "run")
    return U


def diag(U, gamma=5.0 / 3.0, nu=0.0, eta=0.0, cfl=0.1) -> dict:
    U = _fields(U)
    out = np.zeros(len(DIAG_NAMES), dtype=np.float64)
    p = _params(U.shape[1], gamma, nu, eta, 0.0, cfl)
    _check(lib().orc_diag(ctypes.byref(p), _ptr(U), _ptr(out)), "diag")
    return dict(zip(DIAG_NAMES, out.tolist()))


def spectra(U, nshell: int) -> dict:
    """Shell spectra E_u, E_B (nshell shells) and theta', S_3, <(du_x/dx)^2>^(1/2)."""
    U = _fields(U)
    eu, eb, mom = np.zeros(nshell), np.zeros(nshell), np.zeros(3)
    p = _params(U.shape[1])
    _check(lib().orc_spectra(ctypes.byref(p), _ptr(U), int(nshell), _ptr(eu), _ptr(eb), _ptr(mom)), "spectra")
    return {"e_u": eu, "e_b": eb, "theta_rms": mom[0], "s3": mom[1], "dudx_rms": mom[2]}


def cic(f, pos) -> np.ndarray:
    """Cloud-in-cell values (np, nc) of the real fields f (nc, n, n, n) at
    positions pos (np, 3) = (x, y, z)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    nc, n = f.shape[0], f.shape[1]
    out = np.empty((pos.shape[0], nc))
    _check(lib().orc_cic(n, _ptr(f), nc, _ptr(pos), pos.shape[0], _ptr(out)), "cic")
    return out


def tracer_push(B, pos, vel, dt: float, nsteps: int):
    """nsteps Boris steps in the field B (3, n, n, n); returns (pos, vel)."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    vel = np.array(vel, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_tracer_push(B.shape[1], _ptr(B), _ptr(pos), _ptr(vel), pos.shape[0], float(dt), int(nsteps)),
           "tracer_push")
    return pos, vel


def neumaier_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_neumaier_sum(_ptr(x), x.size)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(threads: int) -> None:
    lib().orc_set_num_threads(int(threads))
