"""The launch-class event hooks that bench.py reads (through the C-ABI):
recording leaves the arithmetic untouched, a class mask selects what is
recorded, and the algorithmic bytes agree with the layout of the flux pass
(16 fields in, 12 out, each n^2 rows of K+1 complex values)."""
import numpy as np
import pytest

from paper_1810_12707_amd import inputs as I
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make(n, case):
    from paper_1810_12707_amd.mhd import Solver

    S = Solver(n, "fp32", gamma=case.gamma, nu=case.nu, eta=case.eta, dt=case.dt)
    S.set_state(torch.from_numpy(case.U).to("cuda:0"))
    return S


@pytest.mark.parametrize("n", [32, 48])
def test_profile_hooks(n):
    from paper_1810_12707_amd.mhd import PASS_NAMES

    log(f"[profile] n={n} fp32")
    c = I.random_turbulence(n, b_rms=0.3, seeds=(61, 62, 63))
    A, B = make(n, c), make(n, c)
    A.step(1)
    B.step(1)
    steps = 4
    B.profile(True)
    A.step(steps)
    B.step(steps)
    prof = B.profile_read()
    B.profile(False)
    # recording changes no arithmetic
    assert torch.equal(A.get_state(), B.get_state())
    assert prof["dropped"] == 0
    step_classes = [k for k in PASS_NAMES if k != "reduce"]
    for k in step_classes:
        assert prof[k]["launches"] >= steps, k
        assert prof[k]["ms"] > 0, k
    total = sum(prof[k]["bytes"] for k in PASS_NAMES)
    log(f"  bytes per step {total / steps:.6e}, step_bytes {B.step_bytes:.6e}")
    assert abs(total / steps - B.step_bytes) <= 1e-9 * B.step_bytes
    # flux pass: 28 real-space-in-x arrays of n * n rows of K + 1 complex FP32
    nh = (n - 1) // 3 + 1
    want = 28 * n * n * nh * 8
    log(f"  xb bytes per launch {prof['xb']['bytes'] / prof['xb']['launches']:.0f}, layout {want}")
    assert prof["xb"]["bytes"] == want * prof["xb"]["launches"]
    # a class mask records only its classes
    B.profile(["xb", "zrhs"])
    B.step(2)
    p2 = B.profile_read()
    B.profile(False)
    assert p2["xb"]["launches"] == 2 * prof["xb"]["launches"] // steps
    assert p2["zrhs"]["launches"] == 2 * prof["zrhs"]["launches"] // steps
    assert all(p2[k]["launches"] == 0 for k in PASS_NAMES if k not in ("xb", "zrhs"))
    A.step(2)
    assert torch.equal(A.get_state(), B.get_state())
    A.close()
    B.close()
