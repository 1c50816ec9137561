"""Checkpoint/restart, graph replay and the FP64 CFL status of single runs,
through the C-ABI.

* A run saved after 5 AB2 steps and continued for 5 more in a fresh context
  is bit for bit the uninterrupted 10-step run (the blob carries U^n and the
  history R^{n-1} that the multistep scheme needs, Sections II and IV), also
  when saved before the Euler start.  A flipped byte anywhere in the blob is
  refused with MHD_E_STATE and leaves the context as it was.
* Steps replayed from the captured HIP graph equal steps launched one kernel
  at a time, bit for bit, after every call, with eager work and
  synchronisations between the replays.
* The steps' CFL status is decided on the largest signal speed reduced in
  FP64: on a uniform moving state the speed max|u_i| + c_f is known in closed
  form, and a dt 1e-5 (FP32) or 1e-10 (FP64) below or above the limit is
  accepted or flagged.
"""
import numpy as np
import pytest

from paper_1810_12707_amd import inputs as I
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def solver(n, prec, **kw):
    from paper_1810_12707_amd.mhd import Solver

    return Solver(n, precision=prec, **kw)


def dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype or torch.float64)


def case(n):
    return I.random_turbulence(n, nu=3e-3, eta=4e-3, b_rms=0.3, seeds=(61 + n, 62 + n, 63 + n))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("save_at", [0, 5])
def test_checkpoint_restart_is_bitwise(prec, save_at):
    from paper_1810_12707_amd.mhd import MHD_OK

    n = 32
    log(f"[restart] n={n} prec={prec} save at step {save_at}")
    c = case(n)
    kw = dict(gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt)
    A = solver(n, prec, **kw)
    A.set_state(dev(c.U))
    A.step(10)
    want = A.get_state(torch.float64)
    rc_a, d_a = A.diagnostics()
    A.close()

    B = solver(n, prec, **kw)
    B.set_state(dev(c.U))
    B.step(save_at)
    blob = B.save()
    assert blob.numel() == B.checkpoint_bytes
    B.close()

    C = solver(n, prec, **kw)
    assert C.load(blob) == MHD_OK
    C.step(10 - save_at)
    got = C.get_state(torch.float64)
    rc_c, d_c = C.diagnostics()
    same = bool(torch.equal(got, want))
    log(f"  bitwise equal: {same}; step {d_c['step']} t {d_c['t']:.6e}")
    assert same
    assert rc_c == rc_a == 0 and d_c["step"] == d_a["step"] == 10 and d_c["t"] == d_a["t"]
    C.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_corrupt_or_foreign_blob_is_refused(prec):
    from paper_1810_12707_amd.mhd import MHD_E_ARG, MHD_E_STATE, MHD_OK, MHDError

    n = 24
    log(f"[restart] corrupt blobs n={n} prec={prec}")
    c = case(n)
    kw = dict(gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt)
    S = solver(n, prec, **kw)
    with pytest.raises(MHDError) as e:
        S.save()  # no state yet
    assert e.value.status == MHD_E_STATE
    S.set_state(dev(c.U))
    S.step(3)
    blob = S.save()
    ref_state = S.get_state(torch.float64)
    nbytes = blob.numel()
    rng = np.random.default_rng(7)
    # header bytes (magic, step, checksum word) and payload bytes (state, history, status)
    positions = [0, 26, 250, 256 + 12345 % (nbytes - 300), nbytes // 2 + 3, nbytes - 300]
    positions += [int(p) for p in rng.integers(0, nbytes, 4)]
    for pos in positions:
        bad = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
        off = (-bad.data_ptr()) % 256
        bad = bad[off:off + nbytes]
        bad.copy_(blob)
        bad[pos] ^= 0x10
        T = solver(n, prec, **kw)
        rc = T.load(bad)
        log(f"  flipped byte {pos}: status {rc}")
        assert rc == MHD_E_STATE
        with pytest.raises(MHDError) as e:
            T.step(1)  # the failed load left the context without a state
        assert e.value.status == MHD_E_STATE
        T.close()
    # the intact blob still loads, into a context already holding another state
    T = solver(n, prec, **kw)
    T.set_state(dev(I.random_turbulence(n, seeds=(5, 6, 7)).U))
    T.step(2)
    assert T.load(blob) == MHD_OK
    assert torch.equal(T.get_state(torch.float64), ref_state)
    T.close()
    # a valid blob of another dt is not this run's history
    T = solver(n, prec, **dict(kw, dt=0.5 * c.dt))
    assert T.load(blob) == MHD_E_ARG
    T.close()
    S.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed", "fp64"])
@pytest.mark.parametrize("n", [16, 48])
def test_graph_replay_matches_eager_launches(prec, n):
    from paper_1810_12707_amd.mhd import MHD_FLAG_NO_GRAPH

    log(f"[graph] n={n} prec={prec}")
    c = case(n)
    kw = dict(gamma=c.gamma, nu=c.nu, eta=c.eta, dt=c.dt)
    G = solver(n, prec, **kw)
    E = solver(n, prec, flags=MHD_FLAG_NO_GRAPH, **kw)
    U = dev(c.U)
    G.set_state(U)
    E.set_state(U)
    for k, steps in enumerate((1, 1, 3, 1, 2)):
        G.step(steps)
        E.step(steps)
        a = G.get_state(torch.float64)
        b = E.get_state(torch.float64)
        torch.cuda.synchronize()
        _ = E.diagnostics()  # eager work on the other context between the replays
        same = bool(torch.equal(a, b))
        log(f"  call {k} ({steps} steps): bitwise equal {same}")
        assert same
    G.close()
    E.close()


def uniform_state(n, rho, u0, B0, P0, gamma):
    U = np.zeros((8, n, n, n))
    U[0] = rho
    for i in range(3):
        U[1 + i] = rho * u0[i]
        U[4 + i] = B0[i]
    U[7] = P0 / (gamma - 1) + 0.5 * rho * sum(v * v for v in u0) + 0.5 * sum(b * b for b in B0)
    return U


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_cfl_decision_near_the_limit(prec):
    from paper_1810_12707_amd.mhd import MHD_E_CFL, MHD_FLAG_CHECK_CFL

    n = 16
    gamma, rho, P0 = 5.0 / 3.0, 1.25, 0.8
    u0, B0 = (0.7, 0.1, -0.45), (0.3, -0.2, 0.5)
    U = uniform_state(n, rho, u0, B0, P0, gamma)
    # closed form on the CPU: the fastest signal speed is the same at every point
    speed = max(abs(v) for v in u0) + np.sqrt((gamma * P0 + sum(b * b for b in B0)) / rho)
    cfl = 0.1
    limit = cfl * (2 * np.pi / n) / speed
    margin = 1e-5 if prec == "fp32" else 1e-10
    for f, want in ((1 - margin, 0), (1 + margin, MHD_E_CFL)):
        S = solver(n, prec, gamma=gamma, nu=1e-3, eta=1e-3, dt=f * limit, cfl=cfl, flags=MHD_FLAG_CHECK_CFL)
        S.set_state(dev(U))
        S.step(3)
        rc, d = S.diagnostics()
        log(f"  {prec} dt = {f:.10f} x limit: status {rc}; dt_cfl {d['dt_cfl']:.15e} vs closed form "
            f"{limit:.15e}")
        assert rc == want
        assert abs(d["dt_cfl"] / limit - 1) <= (1e-6 if prec == "fp32" else 1e-13)
        S.close()
