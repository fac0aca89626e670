"""Direct evaluation of eq. (1): f(x_i) = sum_j K(x_i, y_j) s_j.

This is the exact result that the FMM approximates (Section 1).  It is O(MN)
and used only on small inputs or on sampled targets.
"""

import numpy as np

from . import kernel


def _as_2d(charges):
    s = np.asarray(charges, dtype=np.float64)
    return (s[:, None], True) if s.ndim == 1 else (s, False)


def potential(targets, sources, charges, block=2048):
    """phi[i, r] = sum_j K(x_i, y_j) s[j, r]; charges [N] or [N,R]."""
    s, squeeze = _as_2d(charges)
    x = np.asarray(targets, dtype=np.float64)
    out = np.zeros((x.shape[0], s.shape[1]))
    for a in range(0, x.shape[0], block):
        out[a:a + block] = kernel.potential_matrix(x[a:a + block], sources) @ s
    return out[:, 0] if squeeze else out


def gradient(targets, sources, charges, block=1024):
    """grad[i, r, :] = sum_j grad_x K(x_i, y_j) s[j, r]; returns [M,3] or [M,R,3]."""
    s, squeeze = _as_2d(charges)
    x = np.asarray(targets, dtype=np.float64)
    out = np.zeros((x.shape[0], s.shape[1], 3))
    for a in range(0, x.shape[0], block):
        g = kernel.gradient_matrix(x[a:a + block], sources)  # [m, N, 3]
        out[a:a + block] = np.einsum("mnd,nr->mrd", g, s)
    return out[:, 0, :] if squeeze else out


def rel_l2(a, b):
    """Relative L2 error |a - b| / |b| over all entries (Frobenius for gradients)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
