"""kiFMM translation operators of Table 1, built in double precision.

The paper names the operators (S2U, U2U, U2D, D2D, D2T, S2T in Table 1) and
defers their construction to the kernel-independent FMM it builds on
(Section 2.1).  The construction written here, and the readings it rests on:

* Check-to-equivalent maps.  A box's upward-equivalent density u lives on the
  surface at alpha_inner (1.05 r); it is fitted so that its field matches a
  given field on the upward-check surface at alpha_outer (2.95 r):
  u = pinv(K(UC, UE)) * (field on UC).  Downward: d lives on the surface at
  alpha_outer and is fitted to a field on the downward-check surface at
  alpha_inner: d = pinv(K(DC, DE)) * (field on DC).
* Reading (pseudo-inverse): truncated SVD, dropping singular values below
  eps_pinv * sigma_max; as for the compression rank below, the kept count is
  extended so that a cluster of equal singular values is never split.
* All operators are built per level from the actual box radius (no scaling
  identities are used here), in coordinates relative to the box centre, since
  the kernel depends only on x - y.
* U2D (M2L) operator for a target box B and source box A whose centres differ
  by 2 r t (t an integer offset): K(DC_B, UE_A).
* Reading (M2L compression, "BLAS M2L"): stack the U2D matrices of every
  possible V-list offset side by side, [K_1 ... K_m] (n x m n), and on top of
  each other, [K_1; ...; K_m] (m n x n).  The leading k left singular vectors
  of the first give U_k, the leading k right singular vectors of the second
  give V_k, and each operator is replaced by U_k C_t V_k^T with
  C_t = U_k^T K_t V_k.  k counts the singular values of the side-by-side stack
  above eps_svd * sigma_max and is then extended while the next singular value
  (of either stack) lies within a relative 1e-8 of the previous one, so that a
  cluster of equal singular values is never split (the retained subspace is
  then unique).
"""

import itertools

import numpy as np

from . import kernel
from .surface import ALPHA_INNER, ALPHA_OUTER, n_points, reference_surface

CLUSTER_RTOL = 1e-8


def splits_cluster(s, k):
    """True when keeping k singular values would separate s[k] from an equal s[k-1]."""
    return 0 < k < len(s) and (s[k - 1] - s[k]) <= CLUSTER_RTOL * s[k - 1]


def truncated_svd(a, eps):
    """SVD of `a` keeping singular values > eps * sigma_max (whole clusters): returns (U_k, s_k, V_k)."""
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    k = int(np.sum(s > eps * s[0]))
    while splits_cluster(s, k):
        k += 1
    return u[:, :k], s[:k], vt[:k].T


def pinv(a, eps):
    """Truncated-SVD pseudo-inverse V_k diag(1/s_k) U_k^T."""
    u, s, v = truncated_svd(a, eps)
    return (v / s[None, :]) @ u.T


def child_offset(octant, r_child):
    """Centre of child `octant` relative to its parent's centre (x in bit 0, y bit 1, z bit 2)."""
    return np.array([(2 * ((octant >> d) & 1) - 1) * r_child for d in range(3)], dtype=np.float64)


def v_list_offsets():
    """All integer offsets t = (target - source) that a V list can contain, from Table 1's definition.

    Enumerated over the eight positions of a target among its siblings: children of the
    parent's colleagues that are not adjacent to the target.
    """
    offs = set()
    for oc in range(8):
        b = ((oc >> 0) & 1, (oc >> 1) & 1, (oc >> 2) & 1)
        for pc in itertools.product((-1, 0, 1), repeat=3):
            if pc == (0, 0, 0):
                continue
            for ch in range(8):
                a = (2 * pc[0] + (ch & 1), 2 * pc[1] + ((ch >> 1) & 1), 2 * pc[2] + ((ch >> 2) & 1))
                t = (b[0] - a[0], b[1] - a[1], b[2] - a[2])
                if max(abs(v) for v in t) > 1:
                    offs.add(t)
    return sorted(offs)


class Operators:
    """Operators for expansion order p, built lazily per level radius."""

    def __init__(self, p, eps_pinv=1e-7, m2l="plain", eps_svd=1e-7, rank=None,
                 alpha_inner=ALPHA_INNER, alpha_outer=ALPHA_OUTER):
        if m2l not in ("plain", "compressed"):
            raise ValueError("m2l must be 'plain' or 'compressed'")
        self.p = int(p)
        self.n = n_points(self.p)
        self.S = reference_surface(self.p)
        self.eps_pinv = float(eps_pinv)
        self.m2l_mode = m2l
        self.eps_svd = float(eps_svd)
        self.rank = rank
        self.ai = float(alpha_inner)
        self.ao = float(alpha_outer)
        self._cache = {}

    def _memo(self, key, build):
        if key not in self._cache:
            self._cache[key] = build()
        return self._cache[key]

    # --- surfaces relative to a box centre ------------------------------------------------
    def upward_equivalent(self, r, center=(0.0, 0.0, 0.0)):
        return np.asarray(center, dtype=np.float64) + self.ai * r * self.S

    def upward_check(self, r, center=(0.0, 0.0, 0.0)):
        return np.asarray(center, dtype=np.float64) + self.ao * r * self.S

    def downward_equivalent(self, r, center=(0.0, 0.0, 0.0)):
        return np.asarray(center, dtype=np.float64) + self.ao * r * self.S

    def downward_check(self, r, center=(0.0, 0.0, 0.0)):
        return np.asarray(center, dtype=np.float64) + self.ai * r * self.S

    # --- check-to-equivalent maps ---------------------------------------------------------
    def uc2e(self, r):
        """pinv(K(UC, UE)) for a box of half-width r."""
        return self._memo(("uc2e", r), lambda: pinv(
            kernel.potential_matrix(self.upward_check(r), self.upward_equivalent(r)), self.eps_pinv))

    def dc2e(self, r):
        """pinv(K(DC, DE)) for a box of half-width r."""
        return self._memo(("dc2e", r), lambda: pinv(
            kernel.potential_matrix(self.downward_check(r), self.downward_equivalent(r)), self.eps_pinv))

    # --- translations (kernel matrices between surfaces) -----------------------------------
    def m2m_check(self, r_child, octant):
        """K(UC_P, UE_C): field of a child's upward-equivalent density on its parent's upward-check surface."""
        def build():
            return kernel.potential_matrix(self.upward_check(2.0 * r_child),
                                           self.upward_equivalent(r_child, child_offset(octant, r_child)))
        return self._memo(("m2m", r_child, octant), build)

    def l2l_check(self, r_child, octant):
        """K(DC_C, DE_P): field of the parent's downward-equivalent density on a child's downward-check surface."""
        def build():
            return kernel.potential_matrix(self.downward_check(r_child, child_offset(octant, r_child)),
                                           self.downward_equivalent(2.0 * r_child))
        return self._memo(("l2l", r_child, octant), build)

    def m2l_kernel(self, r, t):
        """K(DC_B, UE_A) for boxes of half-width r whose centres differ by c_B - c_A = 2 r t."""
        def build():
            tb = 2.0 * r * np.asarray(t, dtype=np.float64)
            return kernel.potential_matrix(self.downward_check(r, tb), self.upward_equivalent(r))
        return self._memo(("m2lk", r, tuple(t)), build)

    # --- compressed M2L ---------------------------------------------------------------------
    def compression(self, r):
        """(U_k, V_k, {t: C_t}, spectra) for boxes of half-width r (compressed mode)."""
        def build():
            offs = v_list_offsets()
            mats = [kernel.potential_matrix(self.downward_check(r, 2.0 * r * np.asarray(t, dtype=np.float64)),
                                            self.upward_equivalent(r)) for t in offs]
            fat = np.hstack(mats)
            tall = np.vstack(mats)
            uf, sf, _ = np.linalg.svd(fat, full_matrices=False)
            _, st, vtt = np.linalg.svd(tall, full_matrices=False)
            k = self.choose_rank(sf, st)
            uk = uf[:, :k]
            vk = vtt[:k].T
            cores = {t: uk.T @ m @ vk for t, m in zip(offs, mats)}
            return uk, vk, cores, (sf, st)
        return self._memo(("svd", r), build)

    def choose_rank(self, s_fat, s_tall):
        n = len(s_fat)
        if self.rank is not None:
            k = int(self.rank)
        else:
            k = int(np.sum(s_fat > self.eps_svd * s_fat[0]))
        k = max(1, min(k, n))
        while k < n and (splits_cluster(s_fat, k) or splits_cluster(s_tall, k)):
            k += 1
        return k
