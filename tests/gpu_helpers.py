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


def pitch(n):
    """The library's kx pitch of the compact spectrum (K+1 padded)."""
    from paper_1810_12707_amd.mhd import mhd_spectrum_pitch

    return mhd_spectrum_pitch(n)


def compact_from_flat(a, n):
    """Flat interleaved compact spectrum (kx pitch padded) -> [nb][nb][K+1]."""
    K, nb, _ = band(n)
    a = np.asarray(a, dtype=np.float64).reshape(nb, nb, pitch(n), 2)[:, :, :K + 1]
    return a[..., 0] + 1j * a[..., 1]


def flat_from_compact(c, fill=0.0):
    """[nb][nb][K+1] -> flat interleaved with the padded kx pitch; padding set to `fill`."""
    n_b, _, nh = c.shape
    n = 3 * (nh - 1) + 1  # any n with this K gives the same pitch
    out = np.full((n_b, n_b, pitch(n), 2), fill, dtype=np.float64)
    out[:, :, :nh, 0] = c.real
    out[:, :, :nh, 1] = c.imag
    return out.ravel()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def per_field_rel_l2(A, B):
    return [rel_l2(A[f], B[f]) for f in range(A.shape[0])]
