"""Short text summaries of rocprofv3 output, for the profiles/ folder.

    python -m paper_1810_12707_amd.profile_summary stats --csv DIR/x_kernel_stats.csv \
        --command "..." --out profiles/kernels_<workload>.md
    python -m paper_1810_12707_amd.profile_summary traffic --n 256 \
        --fetch DIR/x_counter_collection.csv --write DIR/y_counter_collection.csv \
        --copy-fetch DIR/c_counter_collection.csv --copy-write DIR/d_counter_collection.csv --copy-mib 1024 \
        --command "..." --out profiles/traffic_<workload>.md

`traffic` scales the per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of every
kernel by what the same counters read for a device copy of known size, and
also writes profiles/traffic_<n>.json: HBM bytes per launch of the launch
classes that have a kernel of their own, stamped with a hash of the kernel
sources so that bench.py only reports it while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")


def _code_only(text: str) -> str:
    """C++ source with comments and blank lines removed (comment edits do not
    change the kernels, so they should not invalidate recorded counters)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def source_sha256() -> str:
    """Hash of the code (comments stripped) of every kernel and host source
    file, sorted by name."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def class_kernels(n: int) -> dict:
    """Launch classes whose kernel instance is used by that class alone in a
    step (FP32 path): class -> substring of the demangled kernel name."""
    return {
        "xa": f"k_row<float, {n}, 0, false>",
        "xb": f"k_row<float, {n}, 1, false>",
        "zrhs": f"k_zfwd_rhs<float, {n}, false>",
        "rho": "k_rho_rhs<float>",
    }


def short_name(name: str) -> str:
    name = name.replace("void ", "").replace("mhd::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def cmd_stats(a) -> int:
    with open(a.csv) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# Kernel time: {a.title}", "", "Command (<repo> = the repository root):", "", "```", a.command, "```", "",
             "rocprofv3 `--stats` summary (all kernels of the run, including set-up and diagnostics):", "",
             "| kernel | calls | avg µs | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:a.top]:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}")
    return 0


def per_kernel_kib(path: str, counter: str) -> dict:
    """Mean counter value (KiB) per dispatch of every kernel name."""
    acc = defaultdict(lambda: [0.0, 0])
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            e = acc[r["Kernel_Name"]]
            e[0] += float(r["Counter_Value"])
            e[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


# Launch classes of one step in launch order, with the kernel each uses
# ({mx}: false on the FP32 path, true on the mixed path).
STEP_SEQUENCE = [
    ("zinv_a", "k_col<float, {n}, 1, 1, {mx}, true>"), ("yinv_a", "k_col<float, {n}, 1, 1, {mx}, false>"),
    ("xa", "k_row<float, {n}, 0, {mx}>"), ("yfwd_a", "k_col<float, {n}, -1, 1, {mx}, false>"),
    ("zfwd_a", "k_col<float, {n}, -1, 1, {mx}, true>"), ("zinv_b", "k_col<float, {n}, 1, 3, {mx}, true>"),
    ("yinv_b", "k_col<float, {n}, 1, 1, {mx}, false>"), ("xb", "k_row<float, {n}, 1, {mx}>"),
    ("yfwd_b", "k_col<float, {n}, -1, 1, {mx}, false>"), ("rho", "k_rho_rhs<float>"), ("zrhs", "k_zfwd_rhs<float, {n}, {mx}>"),
]


def per_class_kib(path: str, counter: str, n: int, mixed: bool = False) -> dict:
    """Mean counter value (KiB) per launch class: dispatches are matched to the
    step's fixed launch sequence (steps interrupted by other launches, such as
    diagnostics, are skipped)."""
    recs = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                recs.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    recs.sort()
    mx = "true" if mixed else "false"
    seq = [(c, k.format(n=n, mx=mx)) for c, k in STEP_SEQUENCE]
    acc = defaultdict(lambda: [0.0, 0])
    i = 0
    while i + len(seq) <= len(recs):
        if all(sub in recs[i + t][1] for t, (_, sub) in enumerate(seq)):
            for t, (c, _) in enumerate(seq):
                acc[c][0] += recs[i + t][2]
                acc[c][1] += 1
            i += len(seq)
        else:
            i += 1
    return {c: (v[0] / v[1], v[1]) for c, v in acc.items()}


def copy_factor(path: str, counter: str, mib: int) -> float:
    """Counter reading / true KiB for the largest copy dispatch in the run."""
    d = per_kernel_kib(path, counter)
    best = max(d.values(), key=lambda v: v[0])
    return best[0] / (mib * 1024.0)


def cmd_traffic(a) -> int:
    ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_mib)
    wf = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_mib)
    fetch = per_kernel_kib(a.fetch, "FETCH_SIZE")
    write = per_kernel_kib(a.write, "WRITE_SIZE")
    names = sorted(set(fetch) & set(write), key=lambda k: -(fetch[k][0] / ff + write[k][0] / wf))
    lines = [f"# HBM traffic per dispatch: {a.title}", "", "Commands (<repo> = the repository root; counter passes run one at a time):", "", "```",
             a.command, "```", "",
             f"Calibration on a {a.copy_mib} MiB device copy: FETCH_SIZE reads {ff:.3f}x the true bytes, "
             f"WRITE_SIZE {wf:.3f}x; values below are divided by these factors.", "",
             "| kernel | dispatches | read GB | written GB | total GB |", "|---|---:|---:|---:|---:|"]
    for k in names:
        rd = fetch[k][0] / ff * 1024 / 1e9
        wr = write[k][0] / wf * 1024 / 1e9
        if rd + wr < 1e-3:
            continue
        lines.append(f"| `{short_name(k)}` | {fetch[k][1]} | {rd:.3f} | {wr:.3f} | {rd + wr:.3f} |")
    fc = per_class_kib(a.fetch, "FETCH_SIZE", a.n)
    wc = per_class_kib(a.write, "WRITE_SIZE", a.n)
    alg = {}
    if a.bench_out:
        with open(a.bench_out) as f:
            line = [l for l in f if l.startswith("{")][-1]
        for c, v in json.loads(line)["passes"].items():
            if v.get("GBps"):
                alg[c] = v["GBps"] * v["ms_per_step"] * 1e6  # bytes per launch (one launch per step)
    if fc:
        lines += ["", "Per launch class (dispatches matched to the step's launch sequence):", "",
                  "| class | steps | read GB | written GB | total GB | algorithmic GB | total / algorithmic |",
                  "|---|---:|---:|---:|---:|---:|---:|"]
        for c, _ in STEP_SEQUENCE:
            if c in fc and c in wc:
                rd = fc[c][0] / ff * 1024 / 1e9
                wr = wc[c][0] / wf * 1024 / 1e9
                al = alg.get(c)
                ratio = f"{(rd + wr) / (al / 1e9):.2f}" if al else "-"
                lines.append(f"| {c} | {fc[c][1]} | {rd:.3f} | {wr:.3f} | {rd + wr:.3f} | "
                             f"{al / 1e9 if al else float('nan'):.3f} | {ratio} |")
    out = {}
    for cls, sub in class_kernels(a.n).items():
        hit = [k for k in names if sub in k]
        if len(hit) == 1:
            k = hit[0]
            out[cls] = (fetch[k][0] / ff + write[k][0] / wf) * 1024.0
    rec = {"n": a.n, "source_sha256": source_sha256(), "fetch_factor": ff, "write_factor": wf,
           "bytes_per_launch": out, "command": a.command}
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    jpath = os.path.join(ROOT, "profiles", f"traffic_{a.n}.json")
    with open(jpath, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {a.out} and {jpath}")
    return 0


def cmd_pmc(a) -> int:
    """Mean of every counter in the given runs per launch class."""
    table = {}
    counters = []
    for path in a.csv:
        names = set()
        with open(path) as f:
            for r in csv.DictReader(f):
                names.add(r["Counter_Name"])
        for c in sorted(names):
            counters.append(c)
            table[c] = per_class_kib(path, c, a.n, a.mixed)
    lines = [f"# Hardware counters per launch: {a.title}", "", "Commands (<repo> = the repository root; one pass "
             "per counter group):", "", "```", a.command, "```", "",
             "Mean value per launch of each class (dispatches matched to the step's launch sequence).", "",
             "| class | " + " | ".join(counters) + " |", "|---|" + "---:|" * len(counters)]
    for c, _ in STEP_SEQUENCE:
        vals = []
        for k in counters:
            v = table[k].get(c)
            vals.append(f"{v[0]:.4g}" if v else "-")
        lines.append(f"| {c} | " + " | ".join(vals) + " |")
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}")
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--out", required=True)
    s.add_argument("--top", type=int, default=16)
    s.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--n", type=int, required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--out", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--bench-out", default="", help="stdout of one profiled bench.py run (algorithmic bytes)")
    c = sub.add_parser("pmc")
    c.add_argument("--n", type=int, required=True)
    c.add_argument("--csv", nargs="+", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--out", required=True)
    c.add_argument("--note", default="")
    c.add_argument("--mixed", action="store_true", help="the mixed path's launches (else FP32's)")
    a = ap.parse_args(argv)
    return {"stats": cmd_stats, "traffic": cmd_traffic, "pmc": cmd_pmc}[a.what](a)


if __name__ == "__main__":
    sys.exit(main())
