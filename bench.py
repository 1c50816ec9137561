#!/usr/bin/env python
"""Throughput of the pseudo-spectral compressible-MHD step on one MI355X.

One step = one pass of the hot path: phase A (u^ = D F[m/rho]), phase B
(strain, current, all real-space fluxes, forward transforms, divergence and
curl, resistive term, AB2 update) and the per-step FP64 CFL / non-finite
reduction; the full FP64 diagnostics pass runs every 10 steps inside the timed
region.  Inputs are resident in HBM before timing starts.

Default workload: 256^3 random-phase turbulence (solenoidal u with E(k) ~ k^-2
in shells 1-8, Mach 0.3; B rms 0.1 in shells 1-4; rho = 1 +- 1%), FP32,
nu = eta = 2e-3, dt from CFL 0.1.  Reported beside it: the same workload in
FP64 (the paper's precision) and on the mixed path; a secondary 512^3
ABC-dynamo line (nu = eta = 1e-3) measured the same way; the batched ensemble
(64 runs of 32^3..128^3 in one graph per step) against the same runs advanced
one after another; the errors of the FP32 and mixed runs against FP64 runs
after each workload's own step count (1000 steps at 256^3, 200 at 512^3),
outside the timed region; the practical HBM ceiling (the library's own
streaming copy); and the FP64 CPU oracle on the host as a baseline.  --c5 adds
the 1024^3 Orszag-Tang line (throughput, and errors after 50 steps).

Per precision: warm-up steps, then a few steps with every launch class
bracketed by HIP events (the per-pass table "passes", and which class
dominates), then five timed repeats of the timed steps, during which only the
dominant class's launches are bracketed (its per-launch time gives
"roofline"); "value" is the median repeat.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.  --copy-only runs only the streaming copy (for
calibrating rocprofv3's byte counters against a kernel of known traffic).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
PASS_NAMES = ("zinv_a", "yinv_a", "xa", "yfwd_a", "zfwd_a", "zinv_b", "yinv_b", "xb", "yfwd_b", "zrhs", "rho",
              "reduce")
PASS_KERNELS = {
    "zinv_a": "k_col<float,N,1> (inverse z, 4 fields)",
    "yinv_a": "k_col<float,N,1> (inverse y, 4 fields)",
    "xa": "k_row<float,N,RM_XA>",
    "yfwd_a": "k_col<float,N,-1> (forward y, 3 fields)",
    "zfwd_a": "k_col<float,N,-1> (forward z, 3 fields)",
    "zinv_b": "k_col<float,N,1> (inverse z, 12 outputs)",
    "yinv_b": "k_col<float,N,1> (inverse y, 12 fields)",
    "xb": "k_row<float,N,RM_XB>",
    "yfwd_b": "k_col<float,N,-1> (forward y, 12 fields)",
    "zrhs": "k_zfwd_rhs<float,N>",
    "rho": "k_rho_rhs<float>",
    "reduce": "k_reduce",
}
FIELDS = ("rho", "m_x", "m_y", "m_z", "B_x", "B_y", "B_z", "E")
DIAG_KEYS = ("mass", "e_kin", "e_mag", "e_int", "e_tot", "h_cross", "h_mag", "divb_rms", "j_rms", "dt_cfl")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(name: str):
    from paper_1810_12707_amd import inputs as I

    if name == "turb256":
        return I.config_turb256(256)
    if name == "abc512":
        return I.config_dynamo512(512)
    if name.startswith("turb"):
        return I.random_turbulence(int(name[4:]), name=name)
    if name.startswith("abc"):
        return I.abc_dynamo(int(name[3:]), 1e-3, 1e-3, None, 200, name=name)
    if name.startswith("ot"):
        n = int(name[2:])
        if n >= 512:  # the host recipe takes minutes and n^3 host arrays: build it on the GPU
            import torch

            dtype = torch.float64 if n <= 512 else torch.float32  # 1024^3 has no FP64 path
            return I.orszag_tang_device(torch, n, device="cuda:0", dtype=dtype, name=name)
        return I.orszag_tang(n, name=name)
    raise ValueError(name)


def describe(case, prec="FP32") -> str:
    n = case.n
    if case.name.startswith("turb"):
        return (f"{n}^3 random-phase MHD turbulence, {prec}: solenoidal u E(k)~k^-2 shells 1-8 Mach 0.3, "
                f"B rms 0.1 shells 1-4, rho=1+-1%, gamma=5/3, nu=eta={case.nu:g}, dt={case.dt:.3e} (CFL 0.1), "
                "AB2, 2/3 dealiasing")
    if case.name.startswith("ot"):
        return (f"{n}^3 Orszag-Tang-type start, {prec}: u=(-sin y, sin x, 0), B=(-sin y, sin 2x, 0) plus solenoidal "
                f"shells 1-4 of rms 1e-2 in u and B, rho=25/9, P=5/3, gamma=5/3, nu=eta={case.nu:g}, "
                f"dt={case.dt:.3e} (CFL 0.1), AB2, 2/3 dealiasing")
    return (f"{n}^3 ABC-flow dynamo start, {prec}: rho=1, ABC u (A=B=C=1, k=1), B rms 1e-3 shells 1-4, Mach 0.1, "
            f"gamma=5/3, nu=eta={case.nu:g}, dt={case.dt:.3e} (CFL 0.1), AB2, 2/3 dealiasing")


def upload(case, dtype=None):
    """The case's fields on the GPU, field by field (FP64 unless dtype); a
    case built on the GPU is returned as it is (converted if dtype asks)."""
    import torch

    if torch.is_tensor(case.U):
        return case.U if dtype is None or case.U.dtype == dtype else case.U.to(dtype)
    dtype = dtype or torch.float64
    n = case.n
    U = torch.empty((8, n, n, n), dtype=dtype, device="cuda:0")
    for f in range(8):
        U[f] = torch.from_numpy(case.U[f]).to(device="cuda:0", dtype=dtype)
    return U


def timed_run(case, precision: str, steps: int, warmup: int, repeats: int = 5, diag_every: int = 10,
              prof_steps: int = 10, U=None):
    """warmup steps; prof_steps steps with every launch class bracketed by HIP
    events (the per-pass table, and which class dominates); then `repeats`
    timed blocks of `steps` steps, with events around the dominant class's
    launches only (each event pair costs a few microseconds between
    launches).  ms = the median block."""
    import torch

    from paper_1810_12707_amd.mhd import PASS_NAMES, Solver

    dev = torch.device("cuda:0")
    S = Solver(case.n, precision=precision, gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt, device=dev)
    S.set_state(U if U is not None else upload(case))
    for _ in range(warmup):
        S.step(1)
    S.profile(True)
    S.step(prof_steps)
    prof_all = S.profile_read()
    S.profile(False)
    dom = max((k for k in PASS_NAMES if prof_all[k]["launches"] > 0), key=lambda k: prof_all[k]["ms"])
    torch.cuda.synchronize()
    S.profile([dom])
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps, walls = [], []
    rc_diag = 0
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for k in range(steps):
            S.step(1)
            if diag_every and (k + 1) % diag_every == 0:
                rc_diag, _ = S.diagnostics()
        e1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        reps.append(e0.elapsed_time(e1))
    prof_dom = S.profile_read()
    S.profile(False)
    rc_end, diag = S.diagnostics()
    out = {"ms": statistics.median(reps), "repeats_ms": [round(r, 4) for r in reps], "wall_s": sum(walls),
           "prof": prof_all, "prof_steps": prof_steps, "prof_dom": prof_dom, "dominant": dom, "diag": diag,
           "rc": (rc_diag, rc_end), "total_steps": warmup + prof_steps + repeats * steps,
           "step_bytes": S.step_bytes, "ws_bytes": S.workspace.numel()}
    S.close()
    del S
    torch.cuda.empty_cache()
    return out


def diag_errors(d, ref):
    """Relative differences of the FP64-reduced diagnostics from those of the
    FP64 run (div B in units of the rms current density; absolute for
    quantities that vanish in the reference)."""
    out = {}
    for k in DIAG_KEYS:
        a, b = float(d[k]), float(ref[k])
        if k == "divb_rms":  # rounding-level in both: compare in units of the current density
            out[k] = abs(a - b) / float(ref["j_rms"])
        else:
            out[k] = abs(a - b) / abs(b) if abs(b) > 1e-300 else abs(a - b)
    return out


def rel_errors(a, ref):
    import torch

    return {name: float(torch.linalg.vector_norm(a[f] - ref[f], dtype=torch.float64)
                        / torch.linalg.vector_norm(ref[f], dtype=torch.float64))
            for f, name in enumerate(FIELDS)}


def run_state(case, precision, nsteps, U, out_dtype=None):
    """State (FP64 tensor unless out_dtype) and diagnostics after nsteps steps
    in `precision` (graph-replayed steps after the Euler start), and the wall
    time."""
    import torch

    from paper_1810_12707_amd.mhd import Solver

    S = Solver(case.n, precision=precision, gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt,
               device="cuda:0")
    S.set_state(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(nsteps)
    rc, diag = S.diagnostics()
    secs = time.perf_counter() - t0
    st = S.get_state(out_dtype or torch.float64)
    S.close()
    del S
    torch.cuda.empty_cache()
    return st, diag, rc, secs


def error_leg(case, nsteps, U, precisions=("fp32", "mixed"), ref_precision="fp64"):
    """Per-field relative L2 and diagnostic errors of each precision's run
    against the reference run of the same start after `nsteps` steps (the
    workload's own step count), outside every timed region."""
    import torch

    ref, ref_diag, rc_ref, secs_ref = run_state(case, ref_precision, nsteps, U)
    out = {"steps": nsteps, "reference": ref_precision, "reference_status": rc_ref,
           "reference_seconds": round(secs_ref, 2)}
    for prec in precisions:
        st, diag, rc, secs = run_state(case, prec, nsteps, U)
        out[prec] = {"field_rel_l2": rel_errors(st, ref), "diag_rel": diag_errors(diag, ref_diag), "status": rc,
                     "seconds": round(secs, 2)}
        del st
    del ref
    torch.cuda.empty_cache()
    return out


def rate_line(r, n, steps, bytes_per_step=None):
    sec = r["ms"] * 1e-3
    b = bytes_per_step if bytes_per_step is not None else r["step_bytes"]
    return {"value": round(n ** 3 * steps / sec, 1), "unit": "grid-point-steps/s",
            "ms_per_step": round(r["ms"] / steps, 5), "repeats_ms": r["repeats_ms"], "status": r["rc"],
            "step_hbm": {"alg_bytes_per_step": b, "GBps": round(b / (sec / steps) / 1e9, 1),
                         "frac": round(b / (sec / steps) / 1e9 / HBM_PEAK_GBS, 4)},
            "passes": pass_table(r["prof"], r["prof_steps"])}


def roofline_from(prof_dom: dict, dom: str, traffic: dict | None, ceiling: float | None = None):
    """The dominant class's events from the timed region (prof_dom)."""
    p = prof_dom[dom]
    per_launch_bytes = p["bytes"] / p["launches"]
    per_launch_ms = p["ms"] / p["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    t = None
    if traffic and dom in traffic:
        t = traffic[dom]
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": t, "kernel": PASS_KERNELS[dom],
           "bytes_per_launch": per_launch_bytes, "ms_per_launch": round(per_launch_ms, 5),
           "launches_timed": p["launches"]}
    if ceiling:
        out["copy_ceiling_GBps"] = round(ceiling, 1)
        out["frac_of_copy_ceiling"] = round(achieved / ceiling, 4)
    return out


def pass_table(prof: dict, steps: int):
    out = {}
    for k in PASS_NAMES:
        v = prof[k]
        if v["launches"] == 0:
            continue
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None
        out[k] = {"ms_per_step": round(v["ms"] / steps, 5), "GBps": round(gbs, 1) if gbs else None,
                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
    return out


def load_traffic(n: int):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for the
    current kernel sources (profiles/traffic_<n>.json carries a source hash)."""
    from paper_1810_12707_amd.profile_summary import source_sha256

    path = os.path.join(ROOT, "profiles", f"traffic_{n}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_sha256():
        return None
    return rec.get("bytes_per_launch")


def copy_ceiling(mib: int = 1024, reps: int = 5):
    """Read + write rate of the library's streaming copy (mhd_bench_copy) of
    `mib` MiB: the practical HBM ceiling, median of `reps` copies."""
    import torch

    from paper_1810_12707_amd.mhd import mhd_bench_copy

    nbytes = mib << 20
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    mhd_bench_copy(x, y, stream.cuda_stream)  # warm-up
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mhd_bench_copy(x, y, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ok = bool(torch.equal(x[:1 << 20], y[:1 << 20]))
    del x, y
    torch.cuda.empty_cache()
    ms = statistics.median(times)
    return {"GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4), "MiB": mib, "copied_ok": ok,
            "kernel": "k_stream_copy (mhd_bench_copy)"}


def ensemble_run(count: int, steps: int, warmup: int):
    """The batched ensemble (64 runs: 16 each of 32^3, 64^3, 96^3, 128^3,
    seeds 0-63, nu = eta log-uniform in [1e-3, 1e-2], FP32) advanced by
    mhd_ens_step, against the same runs advanced one after another by
    single contexts (graph-replayed steps, same stream, timed the same way)."""
    import torch

    from paper_1810_12707_amd import inputs as I
    from paper_1810_12707_amd.mhd import Ensemble, Solver

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    cases = I.config_ensemble(count)
    log(f"[bench] ensemble inputs: {count} runs in {time.perf_counter() - t0:.1f} s")
    points = sum(c.n ** 3 for c in cases)
    E = Ensemble([{"n": c.n, "precision": "fp32", "gamma": c.gamma, "nu": c.nu, "eta": c.eta, "dt": c.dt}
                  for c in cases], device=dev)
    for i, c in enumerate(cases):
        E.set_state(i, torch.from_numpy(c.U).to(dev))
    t0 = time.perf_counter()
    E.step(warmup)  # tuning, the Euler start, graph capture
    torch.cuda.synchronize()
    log(f"[bench] ensemble warm-up (tuning + capture) {time.perf_counter() - t0:.2f} s; groups {E.groups()}")
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    E.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ens_ms = e0.elapsed_time(e1)
    rc, st, _ = E.diagnostics()
    check = E.get_state(count - 1)
    groups = E.groups()
    step_bytes = E.step_bytes
    E.close()
    del E
    torch.cuda.empty_cache()
    log(f"[bench] ensemble {ens_ms / steps:.3f} ms/step")

    solos = []
    sched = {g["n"]: g["schedule"] for g in groups}
    for c in cases:
        S = Solver(c.n, precision="fp32", gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt, device=dev)
        S.set_state(torch.from_numpy(c.U).to(dev))
        S.set_schedule(sched[c.n])  # each solo on the kernel schedule tuned for its size
        S.step(warmup)  # the Euler start and the capture of its step graph
        solos.append(S)
    torch.cuda.synchronize()
    e0.record(stream)
    for S in solos:
        S.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    same = bool(torch.equal(check, solos[-1].get_state()))
    for S in solos:
        S.close()
    del solos
    torch.cuda.empty_cache()
    log(f"[bench] sequential {seq_ms / steps:.3f} ms/step; last member bitwise equal: {same}")
    ens_rate = points * steps / (ens_ms * 1e-3)
    seq_rate = points * steps / (seq_ms * 1e-3)
    return {
        "workload": f"{count} independent FP32 runs: 16 each of 32^3, 64^3, 96^3, 128^3 "
                    f"({points / 1e6:.1f} M points), random-phase turbulence seeds 0-{count - 1}, "
                    "nu = eta log-uniform in [1e-3, 1e-2], dt from CFL 0.1 per run, AB2",
        "value": round(ens_rate, 1), "unit": "grid-point-steps/s (sum over runs)",
        "ms_per_step": round(ens_ms / steps, 4), "steps": steps, "warmup": warmup,
        "sequential": {"value": round(seq_rate, 1), "ms_per_step": round(seq_ms / steps, 4),
                       "what": "the same runs, each advanced by its own context one after another, every "
                               "step a replay of that context's captured step graph, on the kernel schedule the "
                               "tuner chose for its size"},
        "speedup_vs_sequential": round(ens_rate / seq_rate, 3),
        "step_hbm": {"alg_bytes_per_step": step_bytes,
                     "GBps": round(step_bytes / (ens_ms * 1e-3 / steps) / 1e9, 1),
                     "frac": round(step_bytes / (ens_ms * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS, 4)},
        "groups": groups, "status": rc, "last_member_bitwise_equal_to_solo": same,
    }


def tracer_leg(case, U, count: int = 1 << 20, steps: int = 50):
    """Tracer particles (Section VI) in the workload's field: `count` particles
    at seeded random positions, their initial velocities interpolated from the
    grid, then one call of `steps` Boris pushes (the field synthesised to real
    space once per call), timed with HIP events."""
    import numpy as np
    import torch

    from paper_1810_12707_amd.mhd import Solver

    S = Solver(case.n, precision="fp32", gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt, device="cuda:0")
    S.set_state(U)
    rng = np.random.default_rng(2024)
    pos = torch.from_numpy(rng.uniform(0.0, 2 * np.pi, size=(count, 3))).to("cuda:0")
    vel = S.tracer_velocity(pos)
    dt = 0.1 * (2 * np.pi / case.n) / max(float(vel.abs().max()), 1e-30)  # a tenth of a cell per step
    S.tracer_push(pos, vel, dt, 2)  # warm-up
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    S.tracer_push(pos, vel, dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    S.close()
    return {"value": round(count * steps / (ms * 1e-3), 1), "unit": "particle-steps/s", "particles": count,
            "steps": steps, "ms": round(ms, 4),
            "what": f"cloud-in-cell gather of B + Boris push (FP64 particles) in the {case.n}^3 FP32 field, one "
                    "call of all steps including the field's synthesis to real space"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 CPU oracle (as it stands) on the host: one warm-up step, then
    per size the time of a 4-step run minus a 1-step run (the set-up
    transforms cancel), divided by 3; at all OpenMP threads for 32^3, 64^3,
    128^3 and at one thread for 32^3, 64^3.  value = the 128^3 all-thread
    rate (grid-point-steps/s)."""
    from oracle import oracle as O
    from paper_1810_12707_amd import inputs as I

    threads_all = O.num_threads()

    def per_step(n, threads):
        O.set_num_threads(threads)
        c = I.random_turbulence(n, seeds=(n, n + 1, n + 2))
        O.run(c.U, 1, c.dt, c.gamma, c.nu, c.eta)  # warm-up
        t0 = time.perf_counter()
        O.run(c.U, 1, c.dt, c.gamma, c.nu, c.eta)
        t1 = time.perf_counter()
        O.run(c.U, 4, c.dt, c.gamma, c.nu, c.eta)
        t4 = time.perf_counter() - t1
        return max((t4 - (t1 - t0)) / 3.0, 1e-9)

    table = []
    t_start = time.perf_counter()
    for n, th in ((32, threads_all), (64, threads_all), (128, threads_all), (32, 1), (64, 1)):
        s = per_step(n, th)
        table.append({"n": n, "threads": th, "s_per_step": round(s, 4), "pt_steps_per_s": round(n ** 3 / s, 1)})
    O.set_num_threads(threads_all)
    top = table[2]
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"value": top["pt_steps_per_s"], "unit": "grid-point-steps/s", "cores": threads_all, "kind": "oracle",
            "sample": "AB2 steps of the random-turbulence recipe (FP64, the oracle's own FFT), 3 timed steps "
                      "after 1 warm-up per size; value at 128^3 on all threads (the 256^3 step takes minutes)",
            "threads_used": threads_all, "nproc": nproc, "cpu_model": cpu_model(), "table": table,
            "seconds": round(time.perf_counter() - t_start, 1)}


def c5_leg(warmup: int = 2, steps: int = 5, err_steps: int = 50):
    """The 1024^3 Orszag-Tang line: FP32 and mixed throughput, the mixed-vs-
    FP32 error after err_steps steps at 1024^3 (no FP64 path holds 1024^3),
    and both against FP64 after the same steps of the same start at 512^3."""
    import torch

    from paper_1810_12707_amd import inputs as I

    out = {}
    t0 = time.perf_counter()
    # built on the GPU mode by mode (the host recipe takes ~10 min and 150 GB at 1024^3)
    case = I.orszag_tang_device(torch, 1024, device="cuda:0", dtype=torch.float32, name="ot1024")
    log(f"[bench] c5 inputs in {time.perf_counter() - t0:.1f} s")
    U = case.U
    out["workload"] = describe(case)
    for prec in ("fp32", "mixed"):
        r = timed_run(case, prec, steps, warmup, repeats=1, U=U)
        out[prec] = rate_line(r, 1024, steps)
        out[prec]["roofline"] = roofline_from(r["prof_dom"], r["dominant"], None, None)
        log(f"[bench] c5 {prec}: {out[prec]['ms_per_step']} ms/step")
    # FP32 states (34 GB each at 1024^3) beside one 116 GB workspace at a time
    s32, _, _, _ = run_state(case, "fp32", err_steps, U, torch.float32)
    smx, _, _, _ = run_state(case, "mixed", err_steps, U, torch.float32)
    out["mixed_vs_fp32_1024"] = {"steps": err_steps, "field_rel_l2": rel_errors(smx, s32)}
    del s32, smx, U
    case.U = None
    torch.cuda.empty_cache()
    # the same start and nu = eta at 512^3, in FP64 on the GPU
    c512 = I.orszag_tang_device(torch, 512, device="cuda:0", dtype=torch.float64, name="ot512")
    log("[bench] c5 512^3 error leg")
    out["vs_fp64_512"] = error_leg(c512, err_steps, c512.U)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5, help="timed blocks of --steps steps; value = the median")
    ap.add_argument("--config", default="turb256", help="turb256 (default), abc512, turbN, abcN, otN")
    ap.add_argument("--secondary", default="abc512", help="second workload reported alongside ('' = none)")
    ap.add_argument("--secondary-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-error", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-fp64-rate", action="store_true")
    ap.add_argument("--error-steps", type=int, default=None,
                    help="steps of the error legs (default: the workload's own, 1000 at 256^3, 200 at 512^3)")
    ap.add_argument("--ensemble-steps", type=int, default=20, help="steps of the batched-ensemble line (0 = none)")
    ap.add_argument("--ensemble-count", type=int, default=64)
    ap.add_argument("--c5", action="store_true", help="add the 1024^3 Orszag-Tang line (minutes, ~110 GB host)")
    ap.add_argument("--no-tracers", dest="tracers", action="store_false", help="skip the tracer-particle line")
    ap.add_argument("--copy-only", action="store_true", help="only the streaming copy (counter calibration)")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2

    ceiling = copy_ceiling()
    log(f"[bench] streaming copy ceiling {ceiling['GBps']} GB/s")
    if a.copy_only:
        print(json.dumps({"copy": ceiling}), flush=True)
        return 0

    log(f"[bench] building input {a.config}")
    case = make_case(a.config)
    n = case.n
    U = upload(case)
    log(f"[bench] n={n} dt={case.dt:.3e}; warmup {a.warmup}, {a.repeats} x {a.steps} timed steps")
    r = timed_run(case, "fp32", a.steps, a.warmup, a.repeats, U=U)
    sec = r["ms"] * 1e-3
    value = n ** 3 * a.steps / sec
    dom = r["dominant"]
    roof = roofline_from(r["prof_dom"], dom, load_traffic(n), ceiling["GBps"])
    step_gbs = r["step_bytes"] / (sec / a.steps) / 1e9
    log(f"[bench] {r['ms'] / a.steps:.4f} ms/step, {value:.4e} pt-steps/s; dominant {dom} {roof['achieved']} GB/s")
    mixed = None
    if not a.no_mixed:
        m = timed_run(case, "mixed", a.steps, a.warmup, a.repeats, U=U)
        mixed = rate_line(m, n, a.steps)
        mixed["roofline"] = roofline_from(m["prof_dom"], m["dominant"], None, ceiling["GBps"])
        mixed["what"] = "FP32 data; radix-16 FFT stages as split-BF16x3 MFMA products, FP32 accumulate"
        log(f"[bench] mixed {mixed['ms_per_step']} ms/step")
    fp64 = None
    if not a.no_fp64_rate:
        d = timed_run(case, "fp64", a.steps, a.warmup, a.repeats, U=U)
        fp64 = rate_line(d, n, a.steps)
        fp64["roofline"] = roofline_from(d["prof_dom"], d["dominant"], None, ceiling["GBps"])
        fp64["what"] = "the paper's precision: FP64 data and arithmetic throughout"
        log(f"[bench] fp64 {fp64['ms_per_step']} ms/step")
    tracers = None
    if a.tracers:
        tracers = tracer_leg(case, U)
        log(f"[bench] tracers {tracers['value']:.3e} particle-steps/s")
    err = None
    if not a.no_fp64_error:
        steps_e = a.error_steps or case.steps
        log(f"[bench] error leg: {steps_e} steps in FP64, FP32, mixed")
        err = error_leg(case, steps_e, U, ("fp32",) if a.no_mixed else ("fp32", "mixed"))
    workload = describe(case)
    del U, case
    torch.cuda.empty_cache()

    secondary = None
    if a.secondary:
        log(f"[bench] secondary workload {a.secondary}")
        c2 = make_case(a.secondary)
        U2 = upload(c2)
        r2 = timed_run(c2, "fp32", a.secondary_steps, 3, a.repeats, U=U2)
        s2 = r2["ms"] * 1e-3
        secondary = rate_line(r2, c2.n, a.secondary_steps)
        secondary.update({"workload": describe(c2), "steps": a.secondary_steps,
                          "roofline": roofline_from(r2["prof_dom"], r2["dominant"], load_traffic(c2.n),
                                                    ceiling["GBps"])})
        if not a.no_mixed:
            m2 = timed_run(c2, "mixed", a.secondary_steps, 3, a.repeats, U=U2)
            secondary["mixed_path"] = rate_line(m2, c2.n, a.secondary_steps)
            secondary["mixed_path"]["roofline"] = roofline_from(m2["prof_dom"], m2["dominant"], None,
                                                                ceiling["GBps"])
        if not a.no_fp64_rate:
            d2 = timed_run(c2, "fp64", a.secondary_steps, 3, min(a.repeats, 3), U=U2)
            secondary["fp64_path"] = rate_line(d2, c2.n, a.secondary_steps)
        if not a.no_fp64_error:
            steps_e = a.error_steps or c2.steps
            log(f"[bench] secondary error leg: {steps_e} steps")
            secondary["errors"] = error_leg(c2, steps_e, U2, ("fp32",) if a.no_mixed else ("fp32", "mixed"))
        log(f"[bench] secondary {secondary['ms_per_step']} ms/step")
        del U2, c2
        torch.cuda.empty_cache()

    ensemble = None
    if a.ensemble_steps > 0:
        log(f"[bench] batched ensemble of {a.ensemble_count} runs")
        ensemble = ensemble_run(a.ensemble_count, a.ensemble_steps, 3)

    c5 = None
    if a.c5:
        log("[bench] 1024^3 Orszag-Tang line")
        c5 = c5_leg()

    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline()
        log(f"[bench] cpu {cpu['value']:.3e} pt-steps/s on {cpu['cores']} threads ({cpu['seconds']} s)")

    out = {
        "metric": "grid-point-steps/s",
        "value": round(value, 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms"] / a.steps, 5),
        "repeats_ms": r["repeats_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "grid": n, "global_batch": 1,
                   "parallelism": "none (1 GPU)", "diagnostics_every": 10,
                   "timing": f"median of {a.repeats} blocks of {a.steps} steps"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "step_hbm": {"alg_bytes_per_step": r["step_bytes"], "GBps": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                     "frac_of_copy_ceiling": round(step_gbs / ceiling["GBps"], 4)},
        "copy_ceiling": ceiling,
        "passes": pass_table(r["prof"], r["prof_steps"]),
        "mixed_path": mixed,
        "fp64_path": fp64,
        "errors": err,
        "tracers": tracers,
        "status": r["rc"],
        "wall_s": round(r["wall_s"], 4),
        "secondary": secondary,
        "ensemble": ensemble,
        "c5": c5,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
