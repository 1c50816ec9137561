#!/usr/bin/env python
"""Throughput of the pseudo-spectral compressible-MHD step on one MI355X.

One step = one pass of the hot path: phase A (u^ = D F[m/rho]), phase B
(strain, current, all real-space fluxes, forward transforms, divergence and
curl, resistive term, AB2 update) and the per-step FP64 CFL / non-finite
reduction; the full FP64 diagnostics pass runs every 10 steps inside the timed
region.  Inputs are resident in HBM before timing starts.

Default workload: 256^3 random-phase turbulence (solenoidal u with E(k) ~ k^-2
in shells 1-8, Mach 0.3; B rms 0.1 in shells 1-4; rho = 1 +- 1%), FP32,
nu = eta = 2e-3, dt from CFL 0.1.  A secondary 512^3 ABC-dynamo line
(nu = eta = 1e-3) is measured the same way and reported under "secondary", and
the batched ensemble (64 runs of 32^3..128^3 in one graph per step) against
the same runs advanced one after another under "ensemble".

Per precision: warm-up steps, then a few steps with every launch class
bracketed by HIP events (the per-pass table "passes", and which class
dominates), then the timed steps, during which only the dominant class's
launches are bracketed (its per-launch time gives "roofline"); each event pair
costs a few microseconds between launches, 5% of a 256^3 step if every launch
had one.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
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
        return I.orszag_tang(int(name[2:]), name=name)
    raise ValueError(name)


def describe(case) -> str:
    n = case.n
    if case.name.startswith("turb"):
        return (f"{n}^3 random-phase MHD turbulence, FP32: solenoidal u E(k)~k^-2 shells 1-8 Mach 0.3, "
                f"B rms 0.1 shells 1-4, rho=1+-1%, gamma=5/3, nu=eta={case.nu:g}, dt={case.dt:.3e} (CFL 0.1), "
                "AB2, 2/3 dealiasing")
    if case.name.startswith("ot"):
        return (f"{n}^3 Orszag-Tang-type start, FP32: u=(-sin y, sin x, 0), B=(-sin y, sin 2x, 0) plus solenoidal "
                f"shells 1-4 of rms 1e-2 in u and B, rho=25/9, P=5/3, gamma=5/3, nu=eta={case.nu:g}, "
                f"dt={case.dt:.3e} (CFL 0.1), AB2, 2/3 dealiasing")
    return (f"{n}^3 ABC-flow dynamo start, FP32: rho=1, ABC u (A=B=C=1, k=1), B rms 1e-3 shells 1-4, Mach 0.1, "
            f"gamma=5/3, nu=eta={case.nu:g}, dt={case.dt:.3e} (CFL 0.1), AB2, 2/3 dealiasing")


FIELDS = ("rho", "m_x", "m_y", "m_z", "B_x", "B_y", "B_z", "E")


def timed_run(case, precision: str, steps: int, warmup: int, diag_every: int = 10, prof_steps: int = 10):
    """warmup steps; prof_steps steps with every launch class bracketed by HIP
    events (the per-pass table, and which class dominates); then the timed
    steps, with events around the dominant class's launches only (each event
    pair costs a few microseconds between launches).  The state stays on the
    GPU; `total_steps` counts every step taken."""
    import torch

    from paper_1810_12707_amd.mhd import PASS_NAMES, Solver

    dev = torch.device("cuda:0")
    U64 = torch.from_numpy(case.U).to(dev)
    S = Solver(case.n, precision=precision, gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt, device=dev)
    S.set_state(U64)
    del U64
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    rc_diag = 0
    for k in range(steps):
        S.step(1)
        if diag_every and (k + 1) % diag_every == 0:
            rc_diag, _ = S.diagnostics()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    prof_dom = S.profile_read()
    S.profile(False)
    rc_end, diag = S.diagnostics()
    out = {"ms": ms, "wall_s": wall, "prof": prof_all, "prof_steps": prof_steps, "prof_dom": prof_dom,
           "dominant": dom, "diag": diag, "rc": (rc_diag, rc_end), "total_steps": warmup + prof_steps + steps,
           "step_bytes": S.step_bytes, "ws_bytes": S.workspace.numel(), "state": S.get_state(torch.float64)}
    S.close()
    del S
    torch.cuda.empty_cache()
    return out


def fp64_state(case, nsteps: int):
    """The FP64 GPU run of the same start, same number of steps: its state and
    diagnostics."""
    import torch

    from paper_1810_12707_amd.mhd import Solver

    dev = torch.device("cuda:0")
    D = Solver(case.n, precision="fp64", gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt, device=dev)
    D.set_state(torch.from_numpy(case.U).to(dev))
    D.step(nsteps)
    st = D.get_state(torch.float64)
    _, diag = D.diagnostics()
    D.close()
    del D
    torch.cuda.empty_cache()
    return st, diag


DIAG_KEYS = ("mass", "e_kin", "e_mag", "e_int", "e_tot", "h_cross", "h_mag", "divb_rms", "j_rms", "dt_cfl")


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

    return {name: float(torch.linalg.vector_norm(a[f] - ref[f]) / torch.linalg.vector_norm(ref[f]))
            for f, name in enumerate(FIELDS)}


def run_gpu(case, steps: int, warmup: int, with_fp64_error: bool = True, with_mixed: bool = True):
    r = timed_run(case, "fp32", steps, warmup)
    mixed = timed_run(case, "mixed", steps, warmup) if with_mixed else None
    ref, ref_diag = fp64_state(case, r["total_steps"]) if with_fp64_error else (None, None)
    r["err_vs_fp64"] = rel_errors(r["state"], ref) if ref is not None else None
    r["diag_err_vs_fp64"] = diag_errors(r["diag"], ref_diag) if ref is not None else None
    if mixed is not None:
        mixed["err_vs_fp64"] = rel_errors(mixed["state"], ref) if ref is not None else None
        mixed["diag_err_vs_fp64"] = diag_errors(mixed["diag"], ref_diag) if ref is not None else None
        del mixed["state"]
    del r["state"], ref
    r["mixed"] = mixed
    return r


def mixed_line(m, n, steps):
    if m is None:
        return None
    sec = m["ms"] * 1e-3
    return {"value": round(n ** 3 * steps / sec, 1), "unit": "grid-point-steps/s",
            "ms_per_step": round(m["ms"] / steps, 5), "err_vs_fp64": m["err_vs_fp64"],
            "diag_err_vs_fp64": m["diag_err_vs_fp64"], "status": m["rc"],
            "step_hbm": {"GBps": round(m["step_bytes"] / (sec / steps) / 1e9, 1),
                         "frac": round(m["step_bytes"] / (sec / steps) / 1e9 / HBM_PEAK_GBS, 4)},
            "passes": pass_table(m["prof"], m["prof_steps"]),
            "what": "FP32 data; radix-16 FFT stages as split-BF16x3 MFMA products, FP32 accumulate"}


def roofline_from(prof_dom: dict, dom: str, traffic: dict | None):
    """The dominant class's events from the timed region (prof_dom)."""
    p = prof_dom[dom]
    per_launch_bytes = p["bytes"] / p["launches"]
    per_launch_ms = p["ms"] / p["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    t = None
    if traffic and dom in traffic:
        t = traffic[dom]
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": t, "kernel": PASS_KERNELS[dom],
            "bytes_per_launch": per_launch_bytes, "ms_per_launch": round(per_launch_ms, 5)}


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


def ensemble_run(count: int, steps: int, warmup: int):
    """The batched ensemble (64 runs: 16 each of 32^3, 64^3, 96^3, 128^3,
    seeds 0-63, nu = eta log-uniform in [1e-3, 1e-2], FP32) advanced by
    mhd_ens_step, against the same runs advanced one after another by
    single contexts (same steps, same stream, timed the same way)."""
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
    for c in cases:
        S = Solver(c.n, precision="fp32", gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt, device=dev)
        S.set_state(torch.from_numpy(c.U).to(dev))
        S.step(warmup)
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
                       "what": "the same runs, each advanced by its own context, one after another"},
        "speedup_vs_sequential": round(ens_rate / seq_rate, 3),
        "step_hbm": {"alg_bytes_per_step": step_bytes,
                     "GBps": round(step_bytes / (ens_ms * 1e-3 / steps) / 1e9, 1),
                     "frac": round(step_bytes / (ens_ms * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS, 4)},
        "groups": groups, "status": rc, "last_member_bitwise_equal_to_solo": same,
    }


def cpu_baseline(n_sample: int = 128):
    """The FP64 CPU oracle (as it stands) on one AB2 step of the same
    random-turbulence recipe at n_sample^3, scaled to grid-point-steps/s."""
    from oracle import oracle as O
    from paper_1810_12707_amd import inputs as I

    c = I.random_turbulence(n_sample)
    t0 = time.perf_counter()
    O.run(c.U, 1, c.dt, c.gamma, c.nu, c.eta)
    dt = time.perf_counter() - t0
    return {"value": round(n_sample ** 3 / dt, 1), "unit": "grid-point-steps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"1 AB2 step (RHS + update) of the random-turbulence recipe at {n_sample}^3, FP64, "
                      f"{dt:.2f} s; the 256^3 step would take minutes"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="turb256", help="turb256 (default), abc512, turbN, abcN, otN")
    ap.add_argument("--secondary", default="abc512", help="second workload reported alongside ('' = none)")
    ap.add_argument("--secondary-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-error", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=20, help="steps of the batched-ensemble line (0 = none)")
    ap.add_argument("--ensemble-count", type=int, default=64)
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2

    log(f"[bench] building input {a.config}")
    case = make_case(a.config)
    log(f"[bench] n={case.n} dt={case.dt:.3e}; warmup {a.warmup}, timed {a.steps} steps")
    r = run_gpu(case, a.steps, a.warmup, with_fp64_error=not a.no_fp64_error, with_mixed=not a.no_mixed)
    n = case.n
    sec = r["ms"] * 1e-3
    value = n ** 3 * a.steps / sec
    dom = r["dominant"]
    roof = roofline_from(r["prof_dom"], dom, load_traffic(n))
    step_gbs = r["step_bytes"] / (sec / a.steps) / 1e9
    log(f"[bench] {r['ms'] / a.steps:.4f} ms/step, {value:.4e} pt-steps/s; dominant {dom} {roof['achieved']} GB/s")
    workload = describe(case)
    del case

    secondary = None
    if a.secondary:
        log(f"[bench] secondary workload {a.secondary}")
        c2 = make_case(a.secondary)
        r2 = run_gpu(c2, a.secondary_steps, 3, with_fp64_error=not a.no_fp64_error, with_mixed=not a.no_mixed)
        s2 = r2["ms"] * 1e-3
        roof2 = roofline_from(r2["prof_dom"], r2["dominant"], load_traffic(c2.n))
        secondary = {
            "workload": describe(c2), "value": c2.n ** 3 * a.secondary_steps / s2, "unit": "grid-point-steps/s",
            "ms_per_step": round(r2["ms"] / a.secondary_steps, 4), "steps": a.secondary_steps,
            "roofline": roof2,
            "step_hbm": {"alg_bytes_per_step": r2["step_bytes"],
                         "GBps": round(r2["step_bytes"] / (s2 / a.secondary_steps) / 1e9, 1),
                         "frac": round(r2["step_bytes"] / (s2 / a.secondary_steps) / 1e9 / HBM_PEAK_GBS, 4)},
            "passes": pass_table(r2["prof"], r2["prof_steps"]),
            "err_vs_fp64": r2["err_vs_fp64"], "diag_err_vs_fp64": r2["diag_err_vs_fp64"], "status": r2["rc"],
            "mixed_path": mixed_line(r2["mixed"], c2.n, a.secondary_steps),
        }
        log(f"[bench] secondary {secondary['ms_per_step']} ms/step")
        del c2

    ensemble = None
    if a.ensemble_steps > 0:
        log(f"[bench] batched ensemble of {a.ensemble_count} runs")
        ensemble = ensemble_run(a.ensemble_count, a.ensemble_steps, 3)

    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline()
        log(f"[bench] cpu {cpu['value']:.3e} pt-steps/s on {cpu['cores']} threads")

    out = {
        "metric": "grid-point-steps/s",
        "value": round(value, 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms"] / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "grid": n, "global_batch": 1,
                   "parallelism": "none (1 GPU)", "diagnostics_every": 10},
        "roofline": roof,
        "cpu_baseline": cpu,
        "step_hbm": {"alg_bytes_per_step": r["step_bytes"], "GBps": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "passes": pass_table(r["prof"], r["prof_steps"]),
        "err_vs_fp64": r["err_vs_fp64"],
        "diag_err_vs_fp64": r["diag_err_vs_fp64"],
        "mixed_path": mixed_line(r["mixed"], n, a.steps),
        "status": r["rc"],
        "wall_s": round(r["wall_s"], 4),
        "secondary": secondary,
        "ensemble": ensemble,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
