"""Host-side checks of the C-ABI library (no GPU needed, no compute calls):
it loads, exports every function include/mhd.h declares, validates
parameters, sizes its workspace, and rejects bad workspaces before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def M():
    from paper_1810_12707_amd import mhd

    if not os.path.exists(mhd.LIBPATH):
        pytest.fail("libmhd.so is not built (run __graft_entry__.build())")
    mhd.lib()
    return mhd


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(M):
    names = declared_functions()
    assert len(names) >= 13
    L = M.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(M.EXPORTED) == names


def test_status_strings(M):
    for code in range(-7, 1):
        assert M.status_string(code) and M.status_string(code) != "unknown status"
    assert M.status_string(-99) == "unknown status"


def test_supported_sizes(M):
    for n in (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512):
        assert M.mhd_supported_size(n, M.MHD_FP64) and M.mhd_supported_size(n, M.MHD_FP32)
    for n in (768, 1024):
        assert M.mhd_supported_size(n, M.MHD_FP32) and not M.mhd_supported_size(n, M.MHD_FP64)
    for n in (0, 7, 10, 20, 100, 2048):
        assert not M.mhd_supported_size(n, M.MHD_FP32)
    assert not M.mhd_supported_size(32, 5)


def test_workspace_sizing(M):
    def ws(n, prec):
        return M.mhd_workspace_bytes(M.make_params(n, prec))

    # grows like n^3 (the kx padding weighs on small n) and doubles (to within the small fixed parts) from FP32 to FP64
    assert ws(256, M.MHD_FP32) > 7 * ws(128, M.MHD_FP32)
    r = ws(128, M.MHD_FP64) / ws(128, M.MHD_FP32)
    assert 1.9 < r < 2.01
    # 512^3 FP32 with all fields resident fits easily in one MI355X (288 GB)
    assert ws(512, M.MHD_FP32) < 20e9
    assert ws(1024, M.MHD_FP32) < 150e9
    # the kx pitch: K+1 rounded up to a multiple of 8 (64-byte FP32 rows)
    assert [M.mhd_spectrum_pitch(n) for n in (32, 64, 256, 512, 1024)] == [16, 24, 88, 176, 344]
    assert M.mhd_spectrum_size(32) == 21 * 21 * 16


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("nu", -1.0), ("eta", -0.1), ("dt", 0.0), ("cfl", 0.0),
                                         ("dt", float("nan")), ("precision", 7), ("scheme", 3), ("scheme", -1),
                                         ("force", float("inf"))])
def test_invalid_params_rejected(M, field, value):
    p = M.make_params(32)
    setattr(p, field, value)
    assert M.mhd_workspace_bytes(p) == 0
    ctx = ctypes.c_void_p()
    assert M.lib().mhd_init(ctypes.byref(p), ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(ctx)) == M.MHD_E_ARG


def test_ensemble_members_take_the_plain_ab2_configuration(M):
    """Ensemble members run AB2 without the Section V variants."""
    ok = M.make_params(32)
    assert M.mhd_ens_workspace_bytes([ok, ok]) > 0
    for kw in (dict(scheme="rk4"), dict(scheme="pc"), dict(force=0.1), dict(flags=M.MHD_FLAG_KINEMATIC),
               dict(flags=M.MHD_FLAG_VISC_LAPLACIAN)):
        bad = M.make_params(32, **kw)
        assert M.mhd_workspace_bytes(bad) > 0  # fine for a single run
        assert M.mhd_ens_workspace_bytes([ok, bad]) == 0


def test_alternative_schedule_exists_only_for_fp32_ensemble_sizes(M):
    L = M.lib()
    ctx = ctypes.c_void_p()
    for n, prec in ((48, M.MHD_FP32), (256, M.MHD_FP32), (32, M.MHD_FP64), (64, M.MHD_MIXED)):
        p = M.make_params(n, prec, flags=M.MHD_FLAG_SCHEDULE_ALT)
        need = M.mhd_workspace_bytes(p)
        # refused before any device work (the workspace pointer is never touched)
        assert L.mhd_init(ctypes.byref(p), ctypes.c_void_p(4096), need, None, ctypes.byref(ctx)) == M.MHD_E_SIZE


def test_bad_size_and_workspace(M):
    L = M.lib()
    ctx = ctypes.c_void_p()
    assert L.mhd_init(ctypes.byref(M.make_params(20)), None, 0, None, ctypes.byref(ctx)) == M.MHD_E_SIZE
    assert L.mhd_init(ctypes.byref(M.make_params(1024, M.MHD_FP64)), None, 0, None,
                      ctypes.byref(ctx)) == M.MHD_E_SIZE
    p = M.make_params(32)
    need = M.mhd_workspace_bytes(p)
    assert L.mhd_init(ctypes.byref(p), None, need, None, ctypes.byref(ctx)) == M.MHD_E_WORKSPACE
    assert L.mhd_init(ctypes.byref(p), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(ctx)) == M.MHD_E_WORKSPACE
    assert L.mhd_init(ctypes.byref(p), ctypes.c_void_p(4096 + 8), need, None, ctypes.byref(ctx)) == M.MHD_E_WORKSPACE
    assert L.mhd_init(ctypes.byref(p), ctypes.c_void_p(4096), need, None, None) == M.MHD_E_ARG


def test_null_context_calls(M):
    L = M.lib()
    assert L.mhd_step(None, 1) == M.MHD_E_ARG
    assert L.mhd_set_state(None, None, 0) == M.MHD_E_ARG
    assert L.mhd_rhs(None, None, None, 0) == M.MHD_E_ARG
    assert L.mhd_diagnostics(None, None) == M.MHD_E_ARG
    assert L.mhd_fft3d(None, 1, None, None) == M.MHD_E_ARG
    assert L.mhd_last_error(None) == b""
    assert L.mhd_ens_step(None, 1) == M.MHD_E_ARG
    assert L.mhd_ens_set_state(None, 0, None, 0) == M.MHD_E_ARG
    assert L.mhd_ens_diagnostics(None, None, None) == M.MHD_E_ARG
    assert L.mhd_ens_num_groups(None) == 0
    assert L.mhd_ens_step_bytes(None) == 0.0
    assert L.mhd_ens_last_error(None) == b""
    assert L.mhd_ens_destroy(None) == M.MHD_OK


def test_ensemble_workspace_and_rejections(M):
    L = M.lib()

    def a256(x):
        return (x + 255) // 256 * 256

    plist = [M.make_params(32), M.make_params(64), M.make_params(32, M.MHD_FP64), M.make_params(32)]
    need = M.mhd_ens_workspace_bytes(plist)
    assert need == sum(a256(M.mhd_workspace_bytes(p)) for p in plist)
    # one invalid member invalidates the ensemble
    bad = list(plist) + [M.make_params(20)]
    assert M.mhd_ens_workspace_bytes(bad) == 0
    arr = M._params_array(plist)
    ens = ctypes.c_void_p()
    assert L.mhd_ens_workspace_bytes(arr, 0) == 0
    assert L.mhd_ens_init(arr, 0, ctypes.c_void_p(4096), need, None, None, ctypes.byref(ens)) == M.MHD_E_ARG
    assert L.mhd_ens_init(arr, len(plist), ctypes.c_void_p(4096), need, None, None, None) == M.MHD_E_ARG
    assert L.mhd_ens_init(M._params_array(bad), len(bad), ctypes.c_void_p(4096), need, None, None,
                          ctypes.byref(ens)) == M.MHD_E_SIZE
    assert L.mhd_ens_init(arr, len(plist), ctypes.c_void_p(4096), need - 1, None, None,
                          ctypes.byref(ens)) == M.MHD_E_WORKSPACE
    assert L.mhd_ens_init(arr, len(plist), ctypes.c_void_p(4096 + 64), need, None, None,
                          ctypes.byref(ens)) == M.MHD_E_WORKSPACE
    assert L.mhd_ens_init(arr, len(plist), None, need, None, None, ctypes.byref(ens)) == M.MHD_E_WORKSPACE


def test_pass_names_match_header(M):
    src = open(os.path.join(ROOT, "include", "mhd.h")).read()
    body = re.search(r"enum\s*\{\s*(MHD_PASS_ZINV_A.*?)\}", src, flags=re.S).group(1)
    names = [t.split("=")[0].strip() for t in body.replace("\n", " ").split(",") if t.strip()]
    assert names[-1] == "MHD_PASS_COUNT"
    assert [n[len("MHD_PASS_"):].lower() for n in names[:-1]] == list(M.PASS_NAMES)
