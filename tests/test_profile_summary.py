"""The rocprofv3 summary tool: launch-class attribution of counter values by
the step's launch sequence, and the copy calibration (CPU only)."""
import csv

from paper_1810_12707_amd import profile_summary as P

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def kernel_names(n):
    return {
        "zinv_a": f"void mhd::k_col<float, {n}, 1, 1, false, true>(mhd::ColArgs<float>)",
        "yinv_a": f"void mhd::k_col<float, {n}, 1, 1, false, false>(mhd::ColArgs<float>)",
        "xa": f"void mhd::k_row<float, {n}, 0, false>(mhd::RowArgs<float>)",
        "yfwd_a": f"void mhd::k_col<float, {n}, -1, 1, false, false>(mhd::ColArgs<float>)",
        "zfwd_a": f"void mhd::k_col<float, {n}, -1, 1, false, true>(mhd::ColArgs<float>)",
        "zinv_b": f"void mhd::k_col<float, {n}, 1, 3, false, true>(mhd::ColArgs<float>)",
        "yinv_b": f"void mhd::k_col<float, {n}, 1, 1, false, false>(mhd::ColArgs<float>)",
        "xb": f"void mhd::k_row<float, {n}, 1, false>(mhd::RowArgs<float>)",
        "yfwd_b": f"void mhd::k_col<float, {n}, -1, 1, false, false>(mhd::ColArgs<float>)",
        "rho": "void mhd::(anonymous namespace)::k_rho_rhs<float>(mhd::RhsArgs<float>)",
        "zrhs": f"void mhd::k_zfwd_rhs<float, {n}, false>(mhd::RhsArgs<float>)",
    }


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, counter, value) in enumerate(rows):
            w.writerow([i + 1, i + 1, "Agent 1", 1, 1, 1, 256, 1, name, 256, 0, 0, 8, 0, 16, counter, value, 0, 1])


def test_class_attribution(tmp_path):
    n = 64
    names = kernel_names(n)
    order = [c for c, _ in P.STEP_SEQUENCE]
    rows = []
    for step in range(2):
        for k, c in enumerate(order):
            rows.append((names[c], "FETCH_SIZE", 100.0 * (k + 1) + step))
        # a diagnostics pass between steps must not be attributed
        rows.append((f"void mhd::k_row<float, {n}, 4, false>(mhd::RowArgs<float>)", "FETCH_SIZE", 7.0))
    path = tmp_path / "c.csv"
    write_csv(path, rows)
    got = P.per_class_kib(str(path), "FETCH_SIZE", n)
    assert set(got) == set(order)
    for k, c in enumerate(order):
        assert got[c] == (100.0 * (k + 1) + 0.5, 2)


def test_copy_factor(tmp_path):
    path = tmp_path / "copy.csv"
    write_csv(path, [("fill", "FETCH_SIZE", 3.0), ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0 * 1024)])
    assert abs(P.copy_factor(str(path), "FETCH_SIZE", 1024) - 0.5) < 1e-12


def test_code_only_ignores_comments_but_not_code():
    from paper_1810_12707_amd.profile_summary import _code_only

    a = "int x = 1;  // one\n/* block\n   comment */\nint y = 2;\n\n"
    b = "// header\nint x = 1;\nint y = 2; /* trailing */\n"
    c = "int x = 1;\nint y = 3;\n"
    assert _code_only(a) == _code_only(b)
    assert _code_only(a) != _code_only(c)
