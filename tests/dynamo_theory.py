"""Linear theory of the kinematic ABC dynamo, written for the tests (not part
of the library or the oracle).

With the velocity held fixed, the magnetic field obeys the linear induction
equation dB/dt = curl(u x B) + eta lap B (the paper's kinematic runs of
Section V-B, density and momentum switched off).  For the
Arnold-Beltrami-Childress flow

    u = (A sin z + C cos y,  B sin x + A cos z,  C sin y + B cos x)

every Fourier mode k of B is coupled only to k +- e_x, k +- e_y, k +- e_z,
so on a truncated set of modes the operator is a sparse matrix:

    dB^(k)/dt = i k x sum_q u^(q) x B^(k - q) - eta |k|^2 B^(k),

with q over the six wavevectors of u.  The truncation used here is the one
of a pseudo-spectral solver with the two-thirds rule on an n^3 grid (each
|k_i| < n / 3): the products u x B of a band-limited B have |k_i| <= n/3 + 1,
below the grid's Nyquist number, so such a solver computes exactly this
Galerkin system.  Mean-free fields stay mean-free (the k = 0 row is zero),
and divergence-free fields stay divergence-free (the right-hand side is a
curl plus the Laplacian of a solenoidal field), so the matrix is written on
two real unit vectors perpendicular to each k and the mean is left out.
The growth rate of a field is the real part of the eigenvalue of largest
real part (its magnetic energy grows at twice that rate).
"""
import numpy as np
import scipy.sparse
import scipy.sparse.linalg


def abc_modes(A=1.0, B=1.0, C=1.0):
    """The six Fourier coefficients u^(q) of the ABC flow with k_f = 1, as
    {q: vector}, q = (qx, qy, qz); sin s = (e^{is} - e^{-is}) / 2i and
    cos s = (e^{is} + e^{-is}) / 2."""
    out = {}

    def add(q, v):
        out[q] = out.get(q, np.zeros(3, complex)) + np.asarray(v, complex)

    # u_x = A sin z + C cos y
    add((0, 0, 1), [A / 2j, 0, 0]); add((0, 0, -1), [-A / 2j, 0, 0])
    add((0, 1, 0), [C / 2, 0, 0]); add((0, -1, 0), [C / 2, 0, 0])
    # u_y = B sin x + A cos z
    add((1, 0, 0), [0, B / 2j, 0]); add((-1, 0, 0), [0, -B / 2j, 0])
    add((0, 0, 1), [0, A / 2, 0]); add((0, 0, -1), [0, A / 2, 0])
    # u_z = C sin y + B cos x
    add((0, 1, 0), [0, 0, C / 2j]); add((0, -1, 0), [0, 0, -C / 2j])
    add((1, 0, 0), [0, 0, B / 2]); add((-1, 0, 0), [0, 0, B / 2])
    return out


def _basis(k):
    """Two real orthonormal vectors perpendicular to k (rows)."""
    k = np.asarray(k, float)
    a = np.array([0.0, 0.0, 1.0]) if abs(k[2]) < abs(k[0]) + abs(k[1]) else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(k, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(k / np.linalg.norm(k), e1)
    return np.stack([e1, e2])


def band_modes(n):
    """The nonzero wavevectors (kx, ky, kz) with every |k_i| < n / 3."""
    K = (n - 1) // 3
    r = np.arange(-K, K + 1)
    kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    k = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    return k[np.any(k != 0, axis=1)], K


def induction_matrix(n, eta, A=1.0, B=1.0, C=1.0):
    """The Galerkin induction operator on the solenoidal, mean-free fields of
    the n^3 two-thirds band, as a sparse complex matrix of order
    2 (number of modes); unknown 2 j + s is the component of B^(k_j) along
    the s-th basis vector of k_j."""
    ks, K = band_modes(n)
    index = {tuple(k): j for j, k in enumerate(ks)}
    E = np.stack([_basis(k) for k in ks])  # (m, 2, 3)
    u = abc_modes(A, B, C)
    rows, cols, vals = [], [], []
    for j, k in enumerate(ks):
        kk = k.astype(float)
        for s in range(2):
            rows.append(2 * j + s); cols.append(2 * j + s); vals.append(-eta * float(kk @ kk))
        for q, uq in u.items():
            p = (k[0] - q[0], k[1] - q[1], k[2] - q[2])
            jp = index.get(p)
            if jp is None:  # outside the band, or the mean
                continue
            # i k x (u_q x b) = i [u_q (k . b) - b (k . u_q)]
            M = 1j * (np.outer(uq, kk) - (kk @ uq) * np.eye(3))
            blk = E[j] @ M @ E[jp].T
            for s in range(2):
                for t in range(2):
                    rows.append(2 * j + s); cols.append(2 * jp + t); vals.append(blk[s, t])
    m = 2 * len(ks)
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, m))


def leading_eigenvalues(n, eta, count=4, A=1.0, B=1.0, C=1.0, tol=1e-10):
    """The count eigenvalues of largest real part, largest first."""
    M = induction_matrix(n, eta, A, B, C)
    w = scipy.sparse.linalg.eigs(M, k=count, which="LR", tol=tol, ncv=max(40, 3 * count),
                                 return_eigenvectors=False)
    return w[np.argsort(-w.real)]


def growth_rate(n, eta, A=1.0, B=1.0, C=1.0):
    """Real part of the leading eigenvalue: the field's growth rate."""
    return float(leading_eigenvalues(n, eta, 2, A, B, C)[0].real)
