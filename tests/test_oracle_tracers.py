"""Pins of the oracle's tracer particles (Section VI): cloud-in-cell
interpolation and the Boris push, against closed forms.

* CIC reproduces a grid field at grid points, constants everywhere, and any
  trilinear function of the coordinates inside a cell (it is the trilinear
  interpolant); its weights are the opposite sub-box volumes over the cell
  volume, so they sum to one.
* Boris in a uniform field B rotates v about B by exactly 2 atan(|B| dt / 2)
  per step (|v| is kept to rounding), and the position is the sum of the
  velocities times dt, wrapped periodically; with B = 0 the motion is a
  straight line.
"""
import numpy as np

from oracle import oracle as O


def test_cic_is_trilinear_interpolation():
    n = 12
    dx = 2 * np.pi / n
    rng = np.random.default_rng(3)
    a = rng.standard_normal(8)
    i = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    f = a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * y * z + a[6] * x * z + a[7] * x * y * z
    # particles strictly inside cells that do not cross the periodic seam
    p = rng.uniform(0.1, n - 1.1, size=(200, 3)) * dx
    got = O.cic(f[None], p)[:, 0]
    s = p / dx  # continuous grid coordinates
    want = (a[0] + a[1] * s[:, 0] + a[2] * s[:, 1] + a[3] * s[:, 2] + a[4] * s[:, 0] * s[:, 1]
            + a[5] * s[:, 1] * s[:, 2] + a[6] * s[:, 0] * s[:, 2] + a[7] * s[:, 0] * s[:, 1] * s[:, 2])
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()
    # at grid points: the grid values, also across the seam
    g = rng.standard_normal((2, n, n, n))
    idx = rng.integers(0, n, size=(50, 3))
    got = O.cic(g, idx[:, ::-1].astype(np.float64) * dx + 0.0)
    want = np.stack([g[c][idx[:, 0], idx[:, 1], idx[:, 2]] for c in range(2)], axis=1)
    assert np.abs(got - want).max() < 1e-12
    # constants everywhere, periodic images included
    assert np.abs(O.cic(np.full((1, n, n, n), 2.5), rng.uniform(-10, 20, size=(100, 3)))[:, 0] - 2.5).max() < 1e-13


def rotate(v, axis, angle):
    """Rodrigues rotation of v about the unit vector axis."""
    return (v * np.cos(angle) + np.cross(axis, v) * np.sin(angle) + axis * np.dot(axis, v) * (1 - np.cos(angle)))


def test_boris_uniform_field_gyration():
    n, dt, steps = 8, 0.07, 40
    B0 = np.array([0.3, -0.5, 0.8])
    B = np.broadcast_to(B0[:, None, None, None], (3, n, n, n)).copy()
    rng = np.random.default_rng(5)
    pos0 = rng.uniform(0, 2 * np.pi, size=(4, 3))
    vel0 = rng.standard_normal((4, 3))
    pos, vel = O.tracer_push(B, pos0, vel0, dt, steps)
    bhat = B0 / np.linalg.norm(B0)
    # q = M = 1: the rotation is clockwise about B (dv/dt = v x B)
    theta = -2 * np.arctan(np.linalg.norm(B0) * dt / 2)
    for p in range(4):
        v = vel0[p].copy()
        x = pos0[p].copy()
        for _ in range(steps):
            v = rotate(v, bhat, theta)
            x = x + v * dt
        assert np.abs(vel[p] - v).max() < 1e-13
        d = (pos[p] - x + np.pi) % (2 * np.pi) - np.pi  # equal modulo the period
        assert np.abs(d).max() < 1e-12
        assert abs(np.linalg.norm(vel[p]) - np.linalg.norm(vel0[p])) < 1e-13
        assert np.all((pos[p] >= 0) & (pos[p] < 2 * np.pi))


def test_boris_free_streaming():
    n = 8
    pos0 = np.array([[6.2, 0.1, 3.0]])
    vel0 = np.array([[0.5, -0.3, 0.25]])
    pos, vel = O.tracer_push(np.zeros((3, n, n, n)), pos0, vel0, 0.1, 7)
    assert np.array_equal(vel, vel0)
    want = (pos0 + 0.7 * vel0) % (2 * np.pi)
    assert np.abs(pos - want).max() < 1e-13
