"""Writes the oracle regression fixtures in this folder.

Calls only the oracle (and the seeded input generator); nothing here comes
from the HIP path.  Re-run after a deliberate change to the oracle's
arithmetic, and name the passage of the paper that justifies the change in the
commit message.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1810_12707_amd import inputs as I  # noqa: E402


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


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_abc16_10steps.json")
    with open(out, "w") as f:
        json.dump(abc16(), f, indent=1, sort_keys=True)
    print("wrote", out)
