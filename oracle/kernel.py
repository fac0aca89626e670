"""Laplace kernel, eq. (2) of Section 1: K(x, y) = 1 / |x - y|.

Reading (kernel normalisation): the paper writes the kernel without the
1/(4 pi) factor, so none is applied.

Reading (coincident points): with sources equal to targets, eq. (1) contains
the singular term j = i.  Every pair with |x - y| = 0 contributes zero to the
potential and to its gradient.
"""

import numpy as np


def potential_matrix(targets, sources):
    """K[i, j] = 1 / |x_i - y_j|, and 0 where x_i == y_j.  Shapes [M,3], [N,3] -> [M,N]."""
    x = np.asarray(targets, dtype=np.float64)
    y = np.asarray(sources, dtype=np.float64)
    diff = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    out = np.zeros_like(r)
    nz = r > 0.0
    out[nz] = 1.0 / r[nz]
    return out


def gradient_matrix(targets, sources):
    """G[i, j, :] = grad_x K(x_i, y_j) = -(x_i - y_j) / |x_i - y_j|^3, and 0 where x_i == y_j.

    Shapes [M,3], [N,3] -> [M,N,3].
    """
    x = np.asarray(targets, dtype=np.float64)
    y = np.asarray(sources, dtype=np.float64)
    diff = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    inv3 = np.zeros_like(r)
    nz = r > 0.0
    inv3[nz] = 1.0 / (r[nz] ** 3)
    return -diff * inv3[:, :, None]
