"""Writes the oracle regression fixtures in this folder.

Calls only the oracle (and the seeded input generator); nothing here comes
from the HIP path.  Re-run after a deliberate change to the oracle's
arithmetic, and name the passage of the paper that justifies the change in the
commit message.

    python tests/golden/make_golden.py            # the 16^3 record (seconds)
    python tests/golden/make_golden.py turb256    # the 256^3 record (minutes, ~13 GB of host memory)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1810_12707_amd import inputs as I  # noqa: E402

# sampled grid points and retained low modes of the 256^3 record
TURB_SAMPLES = 1024
TURB_SAMPLE_SEED = 20181030
TURB_LOW_K = 2


def abc16():
    c = I.config_small(16)
    U = O.run(c.U, 10, c.dt, c.gamma, c.nu, c.eta)
    d = O.diag(U, c.gamma, c.nu, c.eta)
    rms = [float(np.sqrt(np.mean(U[f] ** 2))) for f in range(8)]
    probe = [float(U[f, 3, 5, 7]) for f in range(8)]
    return {
        "what": "oracle state after 10 AB2 steps of the 16^3 ABC-flow dynamo start "
                "(rho = 1, ABC u, seed-0 B rms 1e-3 in shells 1-4, Mach 0.1, nu = eta = 1e-2, dt = 1e-3)",
        "diag": d,
        "field_rms": rms,
        "probe_z3_y5_x7": probe,
    }


def sample_points(n: int, count: int, seed: int) -> np.ndarray:
    """Distinct flat grid indices z*n^2 + y*n + x, sorted (numpy's seeded
    generator; the choice of points carries no arithmetic of the method)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n ** 3, size=count, replace=False))


def low_modes(f: np.ndarray, kmax: int):
    """Unnormalised DFT coefficients f^(k) of a real n^3 field for
    |kx|, |ky|, |kz| <= kmax with kx >= 0, as (kz, ky, kx, re, im) rows."""
    n = f.shape[0]
    F = np.fft.rfftn(f)  # axes (z, y, x); numpy as a library, e^{-i k.x} convention
    rows = []
    for kz in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kx in range(0, kmax + 1):
                v = F[kz % n, ky % n, kx]
                rows.append([kz, ky, kx, float(v.real), float(v.imag)])
    return rows


def turb256(steps: int = 10):
    c = I.config_turb256(256)
    n = c.n
    t0 = time.perf_counter()
    U = O.run(c.U, steps, c.dt, c.gamma, c.nu, c.eta)
    secs = time.perf_counter() - t0
    idx = sample_points(n, TURB_SAMPLES, TURB_SAMPLE_SEED)
    flat = U.reshape(8, -1)
    return {
        "what": f"oracle state after {steps} AB2 steps of the {n}^3 random-phase turbulence start "
                "(solenoidal u with E(k) ~ k^-2 in shells 1-8, rms 1, Mach 0.3; B white in shells 1-4, rms 0.1; "
                "rho = 1 + 1% seeded noise, isentropic P; nu = eta = 2e-3, dt from CFL 0.1)",
        "n": n, "steps": steps, "dt": c.dt, "gamma": c.gamma, "nu": c.nu, "eta": c.eta,
        "oracle_seconds": round(secs, 1), "oracle_threads": O.num_threads(),
        "sample_seed": TURB_SAMPLE_SEED,
        "sample_index": [int(i) for i in idx],
        "samples": [[float(v) for v in flat[f, idx]] for f in range(8)],
        "field_l2": [float(np.sqrt(np.mean(U[f] ** 2))) for f in range(8)],
        "low_k": TURB_LOW_K,
        "low_modes": [low_modes(U[f], TURB_LOW_K) for f in range(8)],
    }


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "abc16"
    if which == "abc16":
        out, rec = os.path.join(HERE, "oracle_abc16_10steps.json"), abc16()
    elif which == "turb256":
        out, rec = os.path.join(HERE, "oracle_turb256_10steps.json"), turb256()
    else:
        raise SystemExit(f"unknown record {which}")
    with open(out, "w") as f:
        json.dump(rec, f, indent=None if which == "turb256" else 1, sort_keys=True)
    print("wrote", out)
