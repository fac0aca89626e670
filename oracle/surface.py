"""kiFMM check and equivalent surfaces.

The paper fixes only the point count of a box's multipole/local representation:
n = 6 (p - 1)^2 + 2 for expansion order p (Section 4, per-process message-size
formula; Section 5 confirms 26 values at p = 3).

Reading (surface geometry): the surface of order p is the set of points of the
regular grid {-1, -1 + 2/(p-1), ..., 1}^3 that lie on the boundary of the cube
[-1, 1]^3, i.e. whose infinity norm is 1.  That set has exactly
p^3 - (p-2)^3 = 6 (p-1)^2 + 2 points.  A box with centre c and half-width r
carries the surface c + alpha * r * S_p.

Reading (radii): upward-equivalent and downward-check surfaces use
alpha_inner = 1.05, upward-check and downward-equivalent surfaces use
alpha_outer = 2.95.  A V-list source box is at least two box widths (4 r) from
the target centre in the infinity norm, and 1.05 + 2.95 = 4, so the target's
downward-check surface never crosses the source's upward-check surface.
"""

import numpy as np

ALPHA_INNER = 1.05
ALPHA_OUTER = 2.95


def n_points(p):
    """Number of surface points for expansion order p (Section 4)."""
    return 6 * (p - 1) ** 2 + 2


def reference_surface(p):
    """S_p: [n, 3] float64 points with infinity norm 1, in lexicographic (i, j, k) grid order.

    Coordinates are (2 i - (p - 1)) / (p - 1): one rounding of an integer ratio, so the
    set is exactly symmetric under x -> -x.
    """
    if p < 2:
        raise ValueError("expansion order p must be >= 2")
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if i in (0, p - 1) or j in (0, p - 1) or k in (0, p - 1):
                    pts.append(((2 * i - (p - 1)) / (p - 1),
                                (2 * j - (p - 1)) / (p - 1),
                                (2 * k - (p - 1)) / (p - 1)))
    return np.array(pts, dtype=np.float64)


def box_surface(p, center, half_width, alpha):
    """The surface c + alpha * r * S_p of a box with centre c and half-width r."""
    return np.asarray(center, dtype=np.float64)[None, :] + alpha * half_width * reference_surface(p)
