"""The shared-memory FMM of Algorithm 1 (Section 2.1), uniform tree, in FP64.

Steps, in the paper's order and notation (Table 1 operators):

(1a) S2U, every leaf beta:   u_beta = S_beta s_beta.  Here S_beta is
     pinv(K(UC, UE)) K(UC, y_beta): the field of the leaf's sources on its
     upward-check surface, fitted by an upward-equivalent density.
(1b) U2U, levels L..3:       u_P += U_{P,beta} u_beta, with
     U_{P,beta} = pinv(K(UC_P, UE_P)) K(UC_P, UE_beta).  The children's fields
     on the parent's check surface are summed first, then fitted once.
(2a) VLI, levels 2..L:       d_beta += T_{beta,alpha} u_alpha for alpha in V(beta),
     with T = pinv(K(DC_beta, DE_beta)) K(DC_beta, UE_alpha).  The algorithm
     listing multiplies by u_beta; the source box's density u_alpha is meant.
(2c) D2D, levels 3..L:       d_beta += D_{beta,P} d_P, with
     D = pinv(K(DC_beta, DE_beta)) K(DC_beta, DE_P).  As in U2U, the VLI and
     D2D contributions are summed as check-surface fields and fitted once.
(3b) D2T, every leaf:        f_beta += E_beta d_beta, E = K(x_beta, DE_beta).
(3c) ULI, every leaf:        f_beta += sum_{alpha in U(beta)} K(x_beta, y_alpha) s_alpha.

Reading (levels): V lists are empty at levels 0 and 1, so (2a) and the downward
densities it seeds exist only at levels 2..L, and (1b) stops at level 2.  With
L <= 1 every pair of leaves is adjacent, and the result is the direct sum.

Gradients follow by applying grad_x K in (3b) and (3c) instead of K.

Reading (compressed M2L): in compressed mode the U2D matrix of offset t is
replaced by U_k C_t V_k^T (see ``operators``).
"""

import numpy as np

from . import kernel, surface
from .tree import Tree


class Result:
    """Potentials, gradients and the per-level densities u, d (dicts keyed by box coordinates)."""

    def __init__(self, phi, grad, u, d):
        self.phi = phi
        self.grad = grad
        self.u = u
        self.d = d


def _charges_2d(tree, charges):
    s = np.asarray(charges, dtype=np.float64)
    squeeze = s.ndim == 1
    if squeeze:
        s = s[:, None]
    if s.shape[0] != tree.points.shape[0]:
        raise ValueError("charges must have one row per point")
    return s, squeeze


def upward_pass(tree, ops, s):
    """Steps (1a) and (1b): upward-equivalent densities u[l][box], levels L..2. s is [N, R]."""
    L = tree.depth
    u = [dict() for _ in range(L + 1)]
    if L < 2:
        return u
    X = tree.points
    rL = tree.radius(L)
    for leaf, idx in tree.leaf_points.items():                       # (1a) S2U
        uc = ops.upward_check(rL, tree.box_center(L, leaf))
        check = kernel.potential_matrix(uc, X[idx]) @ s[idx]
        u[L][leaf] = ops.uc2e(rL) @ check
    for l in range(L, 2, -1):                                         # (1b) U2U
        r = tree.radius(l)
        check = {}
        for box in tree.boxes[l]:
            P = Tree.parent(box)
            contrib = ops.m2m_check(r, Tree.octant(box)) @ u[l][box]
            check[P] = check.get(P, 0.0) + contrib
        for P, c in check.items():
            u[l - 1][P] = ops.uc2e(2.0 * r) @ c
    return u


def m2l_field(tree, ops, l, box, u):
    """Field on the downward-check surface of `box` due to its V list (step (2a))."""
    r = tree.radius(l)
    R = next(iter(u[l].values())).shape[1]
    acc = np.zeros((ops.n, R))
    if ops.m2l_mode == "plain":
        for a in tree.v_list(l, box):
            t = (box[0] - a[0], box[1] - a[1], box[2] - a[2])
            acc += ops.m2l_kernel(r, t) @ u[l][a]
        return acc
    uk, vk, cores, _ = ops.compression(r)
    hat = np.zeros((uk.shape[1], R))
    for a in tree.v_list(l, box):
        t = (box[0] - a[0], box[1] - a[1], box[2] - a[2])
        hat += cores[t] @ (vk.T @ u[l][a])
    return uk @ hat


def downward_pass(tree, ops, u, boxes_needed=None):
    """Steps (2a) and (2c): downward-equivalent densities d[l][box], levels 2..L."""
    L = tree.depth
    d = [dict() for _ in range(L + 1)]
    for l in range(2, L + 1):
        r = tree.radius(l)
        targets = tree.boxes[l] if boxes_needed is None else boxes_needed[l]
        for box in targets:
            check = m2l_field(tree, ops, l, box, u)                  # (2a) VLI
            if l > 2:                                                  # (2c) D2D
                check = check + ops.l2l_check(r, Tree.octant(box)) @ d[l - 1][Tree.parent(box)]
            d[l][box] = ops.dc2e(r) @ check
    return d


def leaf_pass(tree, ops, s, d, leaves, want_grad):
    """Steps (3b) D2T and (3c) ULI for the given leaves. Returns phi [N,R], grad [N,R,3] (NaN elsewhere)."""
    L = tree.depth
    N, R = s.shape
    X = tree.points
    phi = np.full((N, R), np.nan)
    grad = np.full((N, R, 3), np.nan) if want_grad else None
    rL = tree.radius(L)
    for leaf in leaves:
        idx = tree.leaf_points[leaf]
        x = X[idx]
        f = np.zeros((len(idx), R))
        g = np.zeros((len(idx), R, 3)) if want_grad else None
        if L >= 2:                                                     # (3b) D2T
            de = ops.downward_equivalent(rL, tree.box_center(L, leaf))
            f += kernel.potential_matrix(x, de) @ d[L][leaf]
            if want_grad:
                g += np.einsum("mnd,nr->mrd", kernel.gradient_matrix(x, de), d[L][leaf])
        src = np.concatenate([tree.leaf_points[a] for a in tree.u_list(leaf)])   # (3c) ULI
        f += kernel.potential_matrix(x, X[src]) @ s[src]
        if want_grad:
            g += np.einsum("mnd,nr->mrd", kernel.gradient_matrix(x, X[src]), s[src])
        phi[idx] = f
        if want_grad:
            grad[idx] = g
    return phi, grad


def evaluate(tree, ops, charges, gradient=True, target_leaves=None, return_state=False):
    """Algorithm 1 on `tree` with `ops`.

    charges: [N] or [N, R] in input order.  Returns (phi, grad) in input order,
    phi [N] / [N,R], grad [N,3] / [N,R,3] (None when gradient=False).  With
    `target_leaves` (a list of leaf coordinates) the downward and leaf passes
    run only for those leaves and their ancestors; other outputs are NaN.
    """
    s, squeeze = _charges_2d(tree, charges)
    L = tree.depth
    leaves = list(tree.leaf_points) if target_leaves is None else [tuple(b) for b in target_leaves]
    needed = None
    if target_leaves is not None:
        needed = [set() for _ in range(L + 1)]
        for b in leaves:
            for l in range(L, -1, -1):
                needed[l].add((b[0] >> (L - l), b[1] >> (L - l), b[2] >> (L - l)))
        needed = [sorted(x) for x in needed]
    u = upward_pass(tree, ops, s)
    d = downward_pass(tree, ops, u, needed) if L >= 2 else [dict() for _ in range(L + 1)]
    phi, grad = leaf_pass(tree, ops, s, d, leaves, gradient)
    if squeeze:
        phi = phi[:, 0]
        grad = grad[:, 0, :] if grad is not None else None
    if return_state:
        return Result(phi, grad, u, d)
    return phi, grad


def vjp(tree, ops, charges, weights, target_leaves=None):
    """Derivative of the evaluate for the loss L = sum_i w_i f_i, f the potentials
    of densities s at the tree's points (the tree held fixed).

    dL/ds_j = sum_i w_i K(x_i, x_j): since K is symmetric and the sources are the
    targets, this is the evaluate applied to the weights (the adjoint FMM, with
    sources and targets exchanged, is the same operator).

    dL/dx_k = w_k grad f_s(x_k) + s_k grad f_w(x_k): the derivative of f_k through
    its own position plus that of every other f_i through the source at x_k,
    using grad_y K(x, y) = -grad_x K(x, y).

    Returns (grad_charges [N], grad_points [N, 3]) in input order (NaN outside
    `target_leaves` when given).
    """
    s = np.asarray(charges, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    phi, grad = evaluate(tree, ops, np.stack([s, w], axis=1), gradient=True, target_leaves=target_leaves)
    return phi[:, 1], w[:, None] * grad[:, 0, :] + s[:, None] * grad[:, 1, :]


def local_field(tree, ops, charges, state, leaf, x):
    """Potential at arbitrary points x inside `leaf` from the leaf's local density and its U list.

    This is the function the FMM represents inside a leaf (steps (3b) + (3c)); it is
    used to check gradients by finite differences.  charges [N]; returns [M].
    """
    L = tree.depth
    s = np.asarray(charges, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    f = np.zeros(x.shape[0])
    if L >= 2:
        de = ops.downward_equivalent(tree.radius(L), tree.box_center(L, leaf))
        f += kernel.potential_matrix(x, de) @ state.d[L][leaf][:, 0]
    src = np.concatenate([tree.leaf_points[a] for a in tree.u_list(leaf)])
    f += kernel.potential_matrix(x, tree.points[src]) @ s[src]
    return f


def surface_size(p):
    return surface.n_points(p)
