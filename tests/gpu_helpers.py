"""Shared helpers of the GPU tests: compact-spectrum extraction from a full
spectrum, error norms, and a cached solver factory."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def band(n):
    K = (n - 1) // 3
    nb = 2 * K + 1
    idx = np.array([l if l <= K else l - nb for l in range(nb)]) % n
    return K, nb, idx


def compact_from_full(F):
    """Full complex spectrum [kz][ky][kx] -> compact [nb][nb][K+1]."""
    n = F.shape[0]
    K, nb, idx = band(n)
    return F[np.ix_(idx, idx, np.arange(K + 1))]


def compact_from_flat(a, n):
    K, nb, _ = band(n)
    a = np.asarray(a, dtype=np.float64).reshape(nb, nb, K + 1, 2)
    return a[..., 0] + 1j * a[..., 1]


def flat_from_compact(c):
    return np.stack([c.real, c.imag], axis=-1).ravel()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def per_field_rel_l2(A, B):
    return [rel_l2(A[f], B[f]) for f in range(A.shape[0])]
