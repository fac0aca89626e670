"""Pins of the oracle's derivative of the evaluate (oracle.fmm.vjp) against
finite differences in FP64, which share nothing with the formula it uses.

* depth <= 1 (the evaluate is the direct sum): central differences of the
  direct-sum loss L(x, s) = sum_i w_i sum_{j != i} s_j / |x_i - x_j| in every
  charge and in sampled coordinates;
* depth 2 (a real FMM): central differences of the oracle's own loss in the
  charges (L is linear in s, so the difference is exact: (A^T w)_j against the
  formula's (A w)_j, equal up to the FMM's approximation) and in coordinates of
  points away from leaf faces (the tree unchanged).
"""

import numpy as np

from oracle import direct, fmm, operators, tree
from paper_2604_19243_amd import workloads


def _loss_direct(x, s, w):
    return float(w @ direct.potential(x, x, s))


def _loss_fmm(x, s, w, depth, ops):
    t = tree.Tree(x, depth, (0.5, 0.5, 0.5), 0.5)
    phi, _ = fmm.evaluate(t, ops, s, gradient=False)
    return float(w @ phi)


def _setup(n, seed):
    x = workloads.points("cube", n, seed).astype(np.float64)
    s = workloads.charges("uniform11", n, seed + 1).astype(np.float64)
    w = workloads.charges("normal", n, seed + 2).astype(np.float64)
    return x, s, w


def test_vjp_direct_sum_matches_finite_differences():
    x, s, w = _setup(60, 41)
    ops = operators.Operators(3, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
    t = tree.Tree(x, 1, (0.5, 0.5, 0.5), 0.5)
    gs, gx = fmm.vjp(t, ops, s, w)
    h = 1e-6
    fd_s = np.array([(_loss_direct(x, s + h * e, w) - _loss_direct(x, s - h * e, w)) / (2 * h)
                     for e in np.eye(len(s))])
    assert np.max(np.abs(gs - fd_s)) <= 1e-7 * np.max(np.abs(fd_s))
    rng = np.random.default_rng(5)
    for k in rng.choice(len(x), 6, replace=False):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fd = (_loss_direct(xp, s, w) - _loss_direct(xm, s, w)) / (2 * h)
            assert abs(gx[k, c] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.max(np.abs(gx)))


def test_vjp_fmm_matches_finite_differences_of_the_oracle():
    depth, p = 2, 4
    x, s, w = _setup(400, 51)
    ops = operators.Operators(p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
    t = tree.Tree(x, depth, (0.5, 0.5, 0.5), 0.5)
    gs, gx = fmm.vjp(t, ops, s, w)
    scale = np.max(np.abs(gs))
    rng = np.random.default_rng(6)
    h = 1e-3  # L is linear in s: any step gives the exact directional derivative up to rounding
    for j in rng.choice(len(s), 5, replace=False):
        e = np.zeros(len(s))
        e[j] = 1.0
        fd = (_loss_fmm(x, s + h * e, w, depth, ops) - _loss_fmm(x, s - h * e, w, depth, ops)) / (2 * h)
        assert abs(gs[j] - fd) <= 1e-8 * scale
    m = 2 ** depth
    cell = x * m - np.floor(x * m)
    inner = np.where(np.all((cell > 0.05) & (cell < 0.95), axis=1))[0]
    gscale = np.max(np.abs(gx))
    hx = 1e-6
    for k in rng.choice(inner, 4, replace=False):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += hx
            xm[k, c] -= hx
            fd = (_loss_fmm(xp, s, w, depth, ops) - _loss_fmm(xm, s, w, depth, ops)) / (2 * hx)
            assert abs(gx[k, c] - fd) <= 1e-6 * gscale


def test_vjp_is_the_evaluate_of_the_weights_and_a_weighted_field():
    # Two invariants that a dropped term or a swapped weight would break:
    # swapping the roles of s and w leaves grad_points unchanged, and with
    # w = s the charge gradient is the potential of s.
    x, s, w = _setup(300, 61)
    ops = operators.Operators(4, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
    t = tree.Tree(x, 2, (0.5, 0.5, 0.5), 0.5)
    _, gx = fmm.vjp(t, ops, s, w)
    _, gx_swapped = fmm.vjp(t, ops, w, s)
    np.testing.assert_allclose(gx, gx_swapped, rtol=1e-12, atol=1e-12 * np.max(np.abs(gx)))
    gs_self, _ = fmm.vjp(t, ops, s, s)
    phi, _ = fmm.evaluate(t, ops, s, gradient=False)
    np.testing.assert_allclose(gs_self, phi, rtol=1e-12, atol=1e-12 * np.max(np.abs(phi)))
