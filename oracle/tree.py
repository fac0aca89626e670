"""Uniform octree, Morton keys and interaction lists (Section 2.1, Table 1).

The points are enclosed in a cube, which is split into eight octants
recursively down to a user-chosen depth L, so every leaf has the same size
(uniform refinement, Section 2.1).  Level 0 is the root cube and level L holds
the leaves.

Boxes are identified by integer grid coordinates (ix, iy, iz) at their level;
the box at level l containing a leaf with coordinates i has coordinates
i >> (L - l).  Morton keys (Section 2.1: three bits per level, sorted keys are
a pre-order traversal) are used to order points and boxes.

Readings:
* Enclosing cube: the caller passes centre c and half-width R0.  When it does
  not, the cube is centred on the midpoint of the per-axis bounding box and
  R0 = 0.5 * max extent * (1 + 1e-6).
* Leaf assignment: i_d = floor((x_d - (c_d - R0)) / h) with h = 2 R0 / 2^L, in
  double precision, clamped to [0, 2^L - 1] (a point on the top face of the
  cube goes to the last box).
* Morton bit order: bit b of ix, iy, iz goes to key bits 3b, 3b+1, 3b+2.
* Interaction lists (Table 1): a leaf's U list is itself plus its colleagues
  (adjacent boxes at the same level); a box's V list holds the children of its
  parent's colleagues that are not adjacent to it.  Only non-empty boxes are
  kept.  Two boxes at one level are adjacent when their coordinates differ by
  at most 1 on every axis.
"""

import itertools

import numpy as np

OFFSETS_27 = [np.array(o) for o in itertools.product((-1, 0, 1), repeat=3)]


def morton_key(ix, iy, iz, bits):
    """Interleave `bits` low bits of (ix, iy, iz); x in the lowest bit of each triple."""
    key = 0
    for b in range(bits):
        key |= ((int(ix) >> b) & 1) << (3 * b)
        key |= ((int(iy) >> b) & 1) << (3 * b + 1)
        key |= ((int(iz) >> b) & 1) << (3 * b + 2)
    return key


def morton_keys(idx, bits):
    """Vectorised morton_key over an [N,3] integer array."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.zeros(idx.shape[0], dtype=np.uint64)
    one = np.uint64(1)
    for b in range(bits):
        for d in range(3):
            key |= ((idx[:, d] >> np.uint64(b)) & one) << np.uint64(3 * b + d)
    return key


def auto_cube(points):
    """Cube enclosing the points: per-axis bounding-box midpoint, half-width 0.5*max extent*(1+1e-6)."""
    p = np.asarray(points, dtype=np.float64)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    center = 0.5 * (lo + hi)
    half = 0.5 * float(np.max(hi - lo)) * (1.0 + 1e-6)
    if half <= 0.0:
        half = 1.0
    return center, half


def leaf_coordinates(points, depth, center, half_width):
    """Per-point leaf grid coordinates [N,3] int64 (uniform grid of 2^depth boxes per axis)."""
    p = np.asarray(points, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64)
    lo = c - half_width
    h = (2.0 * half_width) / float(2 ** depth)
    idx = np.floor((p - lo[None, :]) / h).astype(np.int64)
    return np.clip(idx, 0, 2 ** depth - 1)


def adjacent(a, b):
    """Boxes at the same level touching (sharing a face, edge or vertex) or equal."""
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]), abs(a[2] - b[2])) <= 1


class Tree:
    """Uniform octree over `points` (sources = targets, Section 2.3)."""

    def __init__(self, points, depth, center=None, half_width=None):
        self.points = np.asarray(points, dtype=np.float64)
        if self.points.ndim != 2 or self.points.shape[1] != 3:
            raise ValueError("points must have shape [N, 3]")
        if depth < 0:
            raise ValueError("depth must be >= 0")
        self.depth = int(depth)
        if center is None or half_width is None:
            center, half_width = auto_cube(self.points)
        self.center = np.asarray(center, dtype=np.float64)
        self.half_width = float(half_width)
        L = self.depth

        self.leaf_index = leaf_coordinates(self.points, L, self.center, self.half_width)
        self.keys = morton_keys(self.leaf_index, L)
        # Stable sort by key: ties keep input order.
        self.order = np.argsort(self.keys, kind="stable")

        # Points of each non-empty leaf, as input indices in sorted order.
        sorted_keys = self.keys[self.order]
        starts = np.flatnonzero(np.r_[True, sorted_keys[1:] != sorted_keys[:-1]])
        ends = np.r_[starts[1:], len(sorted_keys)]
        self.leaf_points = {}
        for a, e in zip(starts, ends):
            b = tuple(int(v) for v in self.leaf_index[self.order[a]])
            self.leaf_points[b] = self.order[a:e].astype(np.int64)

        # Non-empty boxes per level, in Morton order.
        self.boxes = []
        self.nonempty = []
        for l in range(L + 1):
            s = {(b[0] >> (L - l), b[1] >> (L - l), b[2] >> (L - l)) for b in self.leaf_points}
            self.nonempty.append(s)
            self.boxes.append(sorted(s, key=lambda t, l=l: morton_key(t[0], t[1], t[2], l)))

    # --- geometry -----------------------------------------------------------------------
    def radius(self, level):
        """Half-width r_l = R0 / 2^l of a box at `level`."""
        return self.half_width / float(2 ** level)

    def box_center(self, level, box):
        """Centre (c - R0) + (2 i + 1) r_l of box `box` at `level`."""
        r = self.radius(level)
        return (self.center - self.half_width) + (2.0 * np.asarray(box, dtype=np.float64) + 1.0) * r

    # --- relations ----------------------------------------------------------------------
    @staticmethod
    def parent(box):
        return (box[0] >> 1, box[1] >> 1, box[2] >> 1)

    @staticmethod
    def octant(box):
        """Position of a box among its siblings, 0..7 (x in bit 0, y in bit 1, z in bit 2)."""
        return (box[0] & 1) | ((box[1] & 1) << 1) | ((box[2] & 1) << 2)

    @staticmethod
    def children(box):
        return [(2 * box[0] + dx, 2 * box[1] + dy, 2 * box[2] + dz)
                for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]

    def colleagues(self, level, box):
        """Boxes at the same level adjacent to `box`, excluding itself, inside the grid."""
        m = 2 ** level
        out = []
        for o in OFFSETS_27:
            if not o.any():
                continue
            c = (box[0] + int(o[0]), box[1] + int(o[1]), box[2] + int(o[2]))
            if all(0 <= v < m for v in c):
                out.append(c)
        return out

    def u_list(self, leaf):
        """U list of a leaf (Table 1): itself and its colleagues, non-empty ones only."""
        L = self.depth
        cand = [leaf] + self.colleagues(L, leaf)
        return [b for b in cand if b in self.nonempty[L]]

    def v_list(self, level, box):
        """V list (Table 1): children of the parent's colleagues, not adjacent to `box`, non-empty."""
        if level < 2:
            return []
        out = []
        for pc in self.colleagues(level - 1, self.parent(box)):
            for ch in self.children(pc):
                if ch in self.nonempty[level] and not adjacent(ch, box):
                    out.append(ch)
        return out
