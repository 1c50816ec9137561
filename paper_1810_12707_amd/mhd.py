"""Python binding of libmhd (include/mhd.h): argument marshalling only.

Every function keeps the C name and forwards to the HIP library; torch is used
only to own device memory (the workspace and field tensors) and to supply the
stream.  There is no fallback: if libmhd.so is missing or fails to load, the
import of this module's functions raises.

Field tensors are (8, n, n, n) with axes (field, z, y, x), field order
rho, m_x, m_y, m_z, B_x, B_y, B_z, E, dtype float64 or float32, contiguous,
on the GPU the solver was created on.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "_lib", "libmhd.so")

MHD_OK, MHD_E_ARG, MHD_E_SIZE, MHD_E_WORKSPACE, MHD_E_HIP, MHD_E_NONFINITE, MHD_E_CFL, MHD_E_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
MHD_FP64, MHD_FP32, MHD_MIXED = 0, 1, 2
MHD_FLAG_CHECK_CFL = 1
MHD_FLAG_NO_GRAPH = 2
MHD_FLAG_VISC_LAPLACIAN = 4
MHD_FLAG_KINEMATIC = 8
MHD_FLAG_SCHEDULE_ALT = 16
MHD_AB2, MHD_RK4, MHD_PC = 0, 1, 2
SCHEMES = {"ab2": MHD_AB2, "rk4": MHD_RK4, "pc": MHD_PC}

EXPORTED = (
    "mhd_supported_size", "mhd_workspace_bytes", "mhd_init", "mhd_set_state", "mhd_get_state",
    "mhd_rhs", "mhd_step", "mhd_diagnostics", "mhd_fft3d", "mhd_spectrum_size", "mhd_spectrum_pitch", "mhd_destroy",
    "mhd_status_string", "mhd_last_error", "mhd_profile", "mhd_profile_read", "mhd_step_bytes",
    "mhd_checkpoint_bytes", "mhd_save", "mhd_load", "mhd_bench_copy", "mhd_rhs_noalloc",
    "mhd_tracers_velocity", "mhd_tracers_push", "mhd_spectra_shells", "mhd_spectra", "mhd_set_schedule",
    "mhd_ens_workspace_bytes", "mhd_ens_init", "mhd_ens_set_state", "mhd_ens_get_state", "mhd_ens_step",
    "mhd_ens_diagnostics", "mhd_ens_num_groups", "mhd_ens_group_info", "mhd_ens_step_bytes", "mhd_ens_destroy",
    "mhd_ens_last_error",
)

PASS_NAMES = ("zinv_a", "yinv_a", "xa", "yfwd_a", "zfwd_a", "zinv_b", "yinv_b", "xb", "yfwd_b", "zrhs", "rho",
              "reduce")


class mhd_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("gamma", ctypes.c_double), ("nu", ctypes.c_double),
        ("eta", ctypes.c_double), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
        ("force", ctypes.c_double),
    ]


class mhd_diag(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("step", ctypes.c_int64), ("mass", ctypes.c_double),
        ("mom", ctypes.c_double * 3), ("e_kin", ctypes.c_double), ("e_mag", ctypes.c_double),
        ("e_int", ctypes.c_double), ("e_tot", ctypes.c_double), ("h_cross", ctypes.c_double),
        ("h_mag", ctypes.c_double), ("divb_rms", ctypes.c_double), ("divb_max", ctypes.c_double),
        ("divb_rel", ctypes.c_double), ("j_rms", ctypes.c_double), ("dt_cfl", ctypes.c_double),
        ("c_s", ctypes.c_double), ("v_a", ctypes.c_double), ("mach_s", ctypes.c_double),
        ("mach_a", ctypes.c_double), ("nonfinite", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "mom" else v
        return d


class MHDError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmhd.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"libmhd.so not built at {LIBPATH}: run __graft_entry__.build() "
                              "or python -m paper_1810_12707_amd.build_lib")
        L = ctypes.CDLL(LIBPATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER(mhd_params)
        L.mhd_supported_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.mhd_workspace_bytes.argtypes = [P]
        L.mhd_workspace_bytes.restype = ctypes.c_size_t
        L.mhd_init.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.mhd_set_state.argtypes = [vp, vp, ctypes.c_int32]
        L.mhd_get_state.argtypes = [vp, vp, ctypes.c_int32]
        L.mhd_rhs.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.mhd_step.argtypes = [vp, ctypes.c_int32]
        L.mhd_diagnostics.argtypes = [vp, ctypes.POINTER(mhd_diag)]
        L.mhd_fft3d.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.mhd_spectrum_size.argtypes = [ctypes.c_int32]
        L.mhd_spectrum_size.restype = ctypes.c_int64
        L.mhd_spectrum_pitch.argtypes = [ctypes.c_int32]
        L.mhd_spectrum_pitch.restype = ctypes.c_int32
        L.mhd_destroy.argtypes = [vp]
        L.mhd_status_string.argtypes = [ctypes.c_int]
        L.mhd_status_string.restype = ctypes.c_char_p
        L.mhd_last_error.argtypes = [vp]
        L.mhd_last_error.restype = ctypes.c_char_p
        L.mhd_profile.argtypes = [vp, ctypes.c_int32]
        L.mhd_profile.restype = ctypes.c_int
        dp, lp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        L.mhd_profile_read.argtypes = [vp, dp, lp, dp, lp]
        L.mhd_profile_read.restype = ctypes.c_int
        L.mhd_step_bytes.argtypes = [vp]
        L.mhd_step_bytes.restype = ctypes.c_double
        L.mhd_checkpoint_bytes.argtypes = [vp]
        L.mhd_checkpoint_bytes.restype = ctypes.c_size_t
        L.mhd_save.argtypes = [vp, vp]
        L.mhd_bench_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.mhd_rhs_noalloc.argtypes = [P, vp, vp, ctypes.c_int32, vp]
        L.mhd_set_schedule.argtypes = [vp, ctypes.c_int32]
        L.mhd_set_schedule.restype = ctypes.c_int
        L.mhd_spectra_shells.argtypes = [ctypes.c_int32]
        L.mhd_spectra_shells.restype = ctypes.c_int32
        L.mhd_spectra.argtypes = [vp, dp, dp, dp]
        L.mhd_spectra.restype = ctypes.c_int
        L.mhd_tracers_velocity.argtypes = [vp, vp, vp, ctypes.c_int64]
        L.mhd_tracers_velocity.restype = ctypes.c_int
        L.mhd_tracers_push.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32]
        L.mhd_tracers_push.restype = ctypes.c_int
        L.mhd_rhs_noalloc.restype = ctypes.c_int
        L.mhd_bench_copy.restype = ctypes.c_int
        L.mhd_load.argtypes = [vp, vp]
        i32 = ctypes.c_int32
        L.mhd_ens_workspace_bytes.argtypes = [P, i32]
        L.mhd_ens_workspace_bytes.restype = ctypes.c_size_t
        L.mhd_ens_init.argtypes = [P, i32, vp, ctypes.c_size_t, vp, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.mhd_ens_set_state.argtypes = [vp, i32, vp, i32]
        L.mhd_ens_get_state.argtypes = [vp, i32, vp, i32]
        L.mhd_ens_step.argtypes = [vp, i32]
        L.mhd_ens_diagnostics.argtypes = [vp, ctypes.POINTER(mhd_diag), ctypes.POINTER(i32)]
        L.mhd_ens_num_groups.argtypes = [vp]
        L.mhd_ens_num_groups.restype = i32
        ip = ctypes.POINTER(i32)
        L.mhd_ens_group_info.argtypes = [vp, i32, ip, ip, ip, dp, dp, ip]
        L.mhd_ens_step_bytes.argtypes = [vp]
        L.mhd_ens_step_bytes.restype = ctypes.c_double
        L.mhd_ens_destroy.argtypes = [vp]
        L.mhd_ens_last_error.argtypes = [vp]
        L.mhd_ens_last_error.restype = ctypes.c_char_p
        for name in ("mhd_supported_size", "mhd_init", "mhd_set_state", "mhd_get_state", "mhd_rhs",
                     "mhd_step", "mhd_diagnostics", "mhd_fft3d", "mhd_destroy", "mhd_save", "mhd_load",
                     "mhd_ens_init",
                     "mhd_ens_set_state", "mhd_ens_get_state", "mhd_ens_step", "mhd_ens_diagnostics",
                     "mhd_ens_group_info", "mhd_ens_destroy"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().mhd_status_string(int(status)).decode()


def make_params(n, precision=MHD_FP32, gamma=5.0 / 3.0, nu=0.0, eta=0.0, dt=1e-3, cfl=0.1, flags=0,
                scheme=MHD_AB2, force=0.0) -> mhd_params:
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    return mhd_params(int(n), int(precision), int(flags), int(scheme), float(gamma), float(nu), float(eta),
                      float(dt), float(cfl), float(force))


# ---------------------------------------------------------------- same-name wrappers

def mhd_supported_size(n: int, precision: int) -> bool:
    return bool(lib().mhd_supported_size(int(n), int(precision)))


def mhd_workspace_bytes(p: mhd_params) -> int:
    return int(lib().mhd_workspace_bytes(ctypes.byref(p)))


def mhd_spectrum_size(n: int) -> int:
    return int(lib().mhd_spectrum_size(int(n)))


def mhd_spectrum_pitch(n: int) -> int:
    return int(lib().mhd_spectrum_pitch(int(n)))


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.float64:
        return MHD_FP64
    if t.dtype == torch.float32:
        return MHD_FP32
    raise TypeError(f"fields must be float32 or float64, got {t.dtype}")


def _check_fields(t, n: int):
    if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (8, n, n, n):
        raise ValueError(f"expected a contiguous CUDA tensor of shape (8, {n}, {n}, {n}), got "
                         f"{tuple(t.shape)} on {t.device}")


def _rc(rc: int, what: str, ctx=None):
    if rc != MHD_OK:
        msg = what
        if ctx is not None and rc == MHD_E_HIP:
            msg += " [" + lib().mhd_last_error(ctx).decode() + "]"
        raise MHDError(rc, msg)


def mhd_init(p: mhd_params, workspace, stream_handle: int):
    """workspace: uint8 CUDA tensor of >= mhd_workspace_bytes(p) bytes."""
    ctx = ctypes.c_void_p()
    rc = lib().mhd_init(ctypes.byref(p), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                        ctypes.c_void_p(stream_handle), ctypes.byref(ctx))
    _rc(rc, "mhd_init")
    return ctx


def mhd_set_state(ctx, fields):
    _rc(lib().mhd_set_state(ctx, ctypes.c_void_p(fields.data_ptr()), _dtype_code(fields)), "mhd_set_state", ctx)


def mhd_get_state(ctx, out):
    _rc(lib().mhd_get_state(ctx, ctypes.c_void_p(out.data_ptr()), _dtype_code(out)), "mhd_get_state", ctx)


def mhd_rhs(ctx, fields_in, rhs_out):
    if fields_in.dtype != rhs_out.dtype:
        raise TypeError("fields_in and rhs_out must share a dtype")
    _rc(lib().mhd_rhs(ctx, ctypes.c_void_p(fields_in.data_ptr()), ctypes.c_void_p(rhs_out.data_ptr()),
                      _dtype_code(fields_in)), "mhd_rhs", ctx)


def mhd_rhs_noalloc(p: mhd_params, fields_in, rhs_out, stream_handle: int) -> int:
    """Status of the allocation-free right-hand side (MHD_OK, MHD_E_WORKSPACE
    beyond its 64 MiB scratch, ...)."""
    if fields_in.dtype != rhs_out.dtype:
        raise TypeError("fields_in and rhs_out must share a dtype")
    return int(lib().mhd_rhs_noalloc(ctypes.byref(p), ctypes.c_void_p(fields_in.data_ptr()),
                                     ctypes.c_void_p(rhs_out.data_ptr()), _dtype_code(fields_in),
                                     ctypes.c_void_p(stream_handle)))


def mhd_set_schedule(ctx, schedule: int):
    _rc(lib().mhd_set_schedule(ctx, int(schedule)), "mhd_set_schedule", ctx)


def mhd_spectra_shells(n: int) -> int:
    return int(lib().mhd_spectra_shells(int(n)))


def mhd_spectra(ctx, n: int) -> dict:
    ns = mhd_spectra_shells(n)
    eu, eb, mom = (ctypes.c_double * ns)(), (ctypes.c_double * ns)(), (ctypes.c_double * 3)()
    _rc(lib().mhd_spectra(ctx, eu, eb, mom), "mhd_spectra", ctx)
    return {"e_u": list(eu), "e_b": list(eb), "theta_rms": mom[0], "s3": mom[1], "dudx_rms": mom[2]}


def _check_tracers(pos, vel):
    import torch

    for t in (pos, vel):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != 3:
            raise ValueError("tracer arrays must be contiguous float64 CUDA tensors of shape (np, 3)")
    if pos.shape != vel.shape:
        raise ValueError("positions and velocities differ in shape")


def mhd_tracers_velocity(ctx, pos, vel):
    _check_tracers(pos, vel)
    _rc(lib().mhd_tracers_velocity(ctx, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()),
                                   pos.shape[0]), "mhd_tracers_velocity", ctx)


def mhd_tracers_push(ctx, pos, vel, dt: float, nsteps: int):
    _check_tracers(pos, vel)
    _rc(lib().mhd_tracers_push(ctx, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()),
                               pos.shape[0], float(dt), int(nsteps)), "mhd_tracers_push", ctx)


def mhd_step(ctx, nsteps: int):
    _rc(lib().mhd_step(ctx, int(nsteps)), "mhd_step", ctx)


def mhd_diagnostics(ctx) -> tuple[int, dict]:
    d = mhd_diag()
    rc = lib().mhd_diagnostics(ctx, ctypes.byref(d))
    if rc not in (MHD_OK, MHD_E_NONFINITE, MHD_E_CFL):
        _rc(rc, "mhd_diagnostics", ctx)
    return rc, d.as_dict()


def mhd_fft3d(ctx, direction: int, x_in, x_out):
    _rc(lib().mhd_fft3d(ctx, int(direction), ctypes.c_void_p(x_in.data_ptr()), ctypes.c_void_p(x_out.data_ptr())),
        "mhd_fft3d", ctx)


PROFILE_ALL = -1


def mhd_profile(ctx, class_mask):
    """class_mask: bit (1 << i) records launch class PASS_NAMES[i]; True or -1
    records every class; False or 0 stops recording."""
    if class_mask is True:
        class_mask = PROFILE_ALL
    _rc(lib().mhd_profile(ctx, int(class_mask)), "mhd_profile", ctx)


def mhd_profile_read(ctx) -> dict:
    k = len(PASS_NAMES)
    ms, nl, by, dr = (ctypes.c_double * k)(), (ctypes.c_int64 * k)(), (ctypes.c_double * k)(), ctypes.c_int64()
    _rc(lib().mhd_profile_read(ctx, ms, nl, by, ctypes.byref(dr)), "mhd_profile_read", ctx)
    out = {name: {"ms": ms[i], "launches": nl[i], "bytes": by[i]} for i, name in enumerate(PASS_NAMES)}
    out["dropped"] = dr.value
    return out


def mhd_step_bytes(ctx) -> float:
    return float(lib().mhd_step_bytes(ctx))


def mhd_bench_copy(src, dst, stream_handle: int):
    """One streaming copy of src into dst (CUDA tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _rc(lib().mhd_bench_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                             ctypes.c_void_p(stream_handle)), "mhd_bench_copy")


def mhd_checkpoint_bytes(ctx) -> int:
    return int(lib().mhd_checkpoint_bytes(ctx))


def mhd_save(ctx, blob):
    """blob: uint8 CUDA tensor of >= mhd_checkpoint_bytes(ctx) bytes, 256-byte aligned."""
    _rc(lib().mhd_save(ctx, ctypes.c_void_p(blob.data_ptr())), "mhd_save", ctx)


def mhd_load(ctx, blob) -> int:
    """Returns the status (MHD_OK, or MHD_E_STATE / MHD_E_ARG for a blob that
    is not a valid checkpoint of this configuration); raises on other errors."""
    rc = lib().mhd_load(ctx, ctypes.c_void_p(blob.data_ptr()))
    if rc not in (MHD_OK, MHD_E_STATE, MHD_E_ARG):
        _rc(rc, "mhd_load", ctx)
    return rc


def mhd_destroy(ctx):
    lib().mhd_destroy(ctx)


def _rc_ens(rc: int, what: str, ens=None):
    if rc != MHD_OK:
        msg = what
        if ens is not None and rc == MHD_E_HIP:
            msg += " [" + lib().mhd_ens_last_error(ens).decode() + "]"
        raise MHDError(rc, msg)


def _params_array(plist):
    arr = (mhd_params * len(plist))()
    for i, p in enumerate(plist):
        arr[i] = p
    return arr


def mhd_ens_workspace_bytes(plist) -> int:
    return int(lib().mhd_ens_workspace_bytes(_params_array(plist), len(plist)))


def mhd_ens_init(plist, workspace, stream_handle: int, tune_cache_path=None):
    """workspace: uint8 CUDA tensor of >= mhd_ens_workspace_bytes(plist) bytes, 256-byte aligned.
    tune_cache_path: None (tune, keep in memory), "" (no tuning) or a file path."""
    ens = ctypes.c_void_p()
    path = None if tune_cache_path is None else str(tune_cache_path).encode()
    rc = lib().mhd_ens_init(_params_array(plist), len(plist), ctypes.c_void_p(workspace.data_ptr()),
                            workspace.numel(), ctypes.c_void_p(stream_handle), path, ctypes.byref(ens))
    _rc_ens(rc, "mhd_ens_init")
    return ens


def mhd_ens_set_state(ens, member: int, fields):
    _rc_ens(lib().mhd_ens_set_state(ens, int(member), ctypes.c_void_p(fields.data_ptr()), _dtype_code(fields)),
            "mhd_ens_set_state", ens)


def mhd_ens_get_state(ens, member: int, out):
    _rc_ens(lib().mhd_ens_get_state(ens, int(member), ctypes.c_void_p(out.data_ptr()), _dtype_code(out)),
            "mhd_ens_get_state", ens)


def mhd_ens_step(ens, nsteps: int):
    _rc_ens(lib().mhd_ens_step(ens, int(nsteps)), "mhd_ens_step", ens)


def mhd_ens_diagnostics(ens, count: int) -> tuple[int, list[int], list[dict]]:
    d = (mhd_diag * count)()
    st = (ctypes.c_int32 * count)()
    rc = lib().mhd_ens_diagnostics(ens, d, st)
    if rc not in (MHD_OK, MHD_E_NONFINITE, MHD_E_CFL):
        _rc_ens(rc, "mhd_ens_diagnostics", ens)
    return rc, list(st), [d[i].as_dict() for i in range(count)]


def mhd_ens_num_groups(ens) -> int:
    return int(lib().mhd_ens_num_groups(ens))


def mhd_ens_group_info(ens, g: int) -> dict:
    n, pr, nm, sc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    cs, rs = ctypes.c_double(), ctypes.c_double()
    _rc_ens(lib().mhd_ens_group_info(ens, int(g), ctypes.byref(n), ctypes.byref(pr), ctypes.byref(nm),
                                     ctypes.byref(cs), ctypes.byref(rs), ctypes.byref(sc)), "mhd_ens_group_info", ens)
    return {"n": n.value, "precision": pr.value, "members": nm.value, "col_scale": cs.value, "row_scale": rs.value,
            "schedule": sc.value}


def mhd_ens_step_bytes(ens) -> float:
    return float(lib().mhd_ens_step_bytes(ens))


def mhd_ens_destroy(ens):
    lib().mhd_ens_destroy(ens)


# ---------------------------------------------------------------- convenience owners

class Solver:
    """Owns one context, its workspace tensor and the stream it runs on."""

    def __init__(self, n, precision="fp32", gamma=5.0 / 3.0, nu=0.0, eta=0.0, dt=1e-3, cfl=0.1,
                 flags=0, device="cuda:0", stream=None, scheme=MHD_AB2, force=0.0):
        import torch

        self.torch = torch
        self.n = int(n)
        codes = {"fp64": MHD_FP64, "fp32": MHD_FP32, "mixed": MHD_MIXED}
        self.precision = codes[precision] if isinstance(precision, str) else int(precision)
        self.params = make_params(n, self.precision, gamma, nu, eta, dt, cfl, flags, scheme, force)
        nbytes = mhd_workspace_bytes(self.params)
        if nbytes == 0:
            raise MHDError(MHD_E_ARG if mhd_supported_size(n, self.precision) else MHD_E_SIZE, "mhd_workspace_bytes")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = mhd_init(self.params, self._ws, self.stream.cuda_stream)
        self.real_dtype = torch.float64 if self.precision == MHD_FP64 else torch.float32

    @property
    def spectrum_size(self) -> int:
        return mhd_spectrum_size(self.n)

    def set_state(self, U):
        _check_fields(U, self.n)
        mhd_set_state(self.ctx, U)

    def get_state(self, dtype=None):
        out = self.torch.empty((8, self.n, self.n, self.n), dtype=dtype or self.torch.float64, device=self.device)
        mhd_get_state(self.ctx, out)
        return out

    def rhs(self, U):
        _check_fields(U, self.n)
        out = self.torch.empty_like(U)
        mhd_rhs(self.ctx, U, out)
        return out

    def step(self, nsteps=1):
        mhd_step(self.ctx, nsteps)

    def diagnostics(self) -> tuple[int, dict]:
        return mhd_diagnostics(self.ctx)

    @property
    def spectrum_pitch(self) -> int:
        return mhd_spectrum_pitch(self.n)

    def fft_forward(self, f):
        """Real n^3 field (working precision) -> compact spectrum (flat, interleaved,
        kx pitch `spectrum_pitch`; padding entries are left unwritten)."""
        n = self.n
        assert f.is_cuda and f.is_contiguous() and tuple(f.shape) == (n, n, n) and f.dtype == self.real_dtype
        out = self.torch.zeros(2 * self.spectrum_size, dtype=self.real_dtype, device=self.device)
        mhd_fft3d(self.ctx, -1, f, out)
        return out

    def fft_inverse(self, spec):
        n = self.n
        assert spec.is_cuda and spec.is_contiguous() and spec.numel() == 2 * self.spectrum_size
        out = self.torch.empty((n, n, n), dtype=self.real_dtype, device=self.device)
        mhd_fft3d(self.ctx, 1, spec, out)
        return out

    def profile(self, enable=True):
        """enable: True (every launch class), False, a bit mask, or a list of pass names."""
        if isinstance(enable, (list, tuple)):
            enable = sum(1 << PASS_NAMES.index(name) for name in enable)
        mhd_profile(self.ctx, enable)

    def profile_read(self) -> dict:
        return mhd_profile_read(self.ctx)

    @property
    def step_bytes(self) -> float:
        return mhd_step_bytes(self.ctx)

    def set_schedule(self, schedule: int):
        """Kernel schedule of later steps (0 default, 1 the alternative build)."""
        mhd_set_schedule(self.ctx, schedule)

    def spectra(self) -> dict:
        """Section V turbulence diagnostics of the current state (see mhd_spectra)."""
        return mhd_spectra(self.ctx, self.n)

    def tracer_velocity(self, pos):
        """Grid velocity at the tracer positions pos (np, 3) float64 CUDA."""
        vel = self.torch.empty_like(pos)
        mhd_tracers_velocity(self.ctx, pos, vel)
        return vel

    def tracer_push(self, pos, vel, dt, nsteps=1):
        """Boris-push the tracers in place through nsteps steps of dt."""
        mhd_tracers_push(self.ctx, pos, vel, dt, nsteps)

    @property
    def checkpoint_bytes(self) -> int:
        return mhd_checkpoint_bytes(self.ctx)

    def save(self):
        """A new checkpoint blob (uint8 CUDA tensor view, 256-byte aligned)."""
        nbytes = self.checkpoint_bytes
        raw = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        blob = raw[off:off + nbytes]
        mhd_save(self.ctx, blob)
        return blob

    def load(self, blob) -> int:
        return mhd_load(self.ctx, blob)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            mhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Owns one ensemble: its workspace tensor, the stream it runs on and the
    member parameters (a list of dicts with keys n, precision, gamma, nu, eta,
    dt, cfl, flags; missing keys take make_params' defaults)."""

    def __init__(self, members, device="cuda:0", stream=None, tune_cache=None):
        import torch

        self.torch = torch
        codes = {"fp64": MHD_FP64, "fp32": MHD_FP32, "mixed": MHD_MIXED}
        self.plist = []
        for m in members:
            m = dict(m)
            pr = m.pop("precision", MHD_FP32)
            m["precision"] = codes[pr] if isinstance(pr, str) else int(pr)
            self.plist.append(make_params(**m))
        self.count = len(self.plist)
        nbytes = mhd_ens_workspace_bytes(self.plist)
        if nbytes == 0:
            raise MHDError(MHD_E_ARG, "mhd_ens_workspace_bytes")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ens = mhd_ens_init(self.plist, self._ws, self.stream.cuda_stream, tune_cache)

    def n_of(self, member: int) -> int:
        return int(self.plist[member].n)

    def set_state(self, member: int, U):
        _check_fields(U, self.n_of(member))
        mhd_ens_set_state(self.ens, member, U)

    def get_state(self, member: int, dtype=None):
        n = self.n_of(member)
        out = self.torch.empty((8, n, n, n), dtype=dtype or self.torch.float64, device=self.device)
        mhd_ens_get_state(self.ens, member, out)
        return out

    def step(self, nsteps=1):
        mhd_ens_step(self.ens, nsteps)

    def diagnostics(self):
        return mhd_ens_diagnostics(self.ens, self.count)

    def groups(self) -> list[dict]:
        return [mhd_ens_group_info(self.ens, g) for g in range(mhd_ens_num_groups(self.ens))]

    @property
    def step_bytes(self) -> float:
        return mhd_ens_step_bytes(self.ens)

    def close(self):
        if getattr(self, "ens", None) is not None:
            mhd_ens_destroy(self.ens)
            self.ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
