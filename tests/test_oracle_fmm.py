"""Pins of the oracle's FMM (Algorithm 1) against the direct sum and exact properties."""

import numpy as np
import pytest

from oracle import direct, fmm, operators, tree
from paper_2604_19243_amd import workloads


def _small(n=2000, seed=21):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)).astype(np.float32).astype(np.float64)
    s = rng.random(n)
    return x, s


@pytest.mark.parametrize("depth", [0, 1])
def test_shallow_tree_is_exactly_the_direct_sum(depth):
    # At depth <= 1 every leaf is adjacent to every other (Table 1), so the FMM is eq. (1).
    x, s = _small(1500)
    t = tree.Tree(x, depth, (0.5, 0.5, 0.5), 0.5)
    phi, g = fmm.evaluate(t, operators.Operators(4), s)
    np.testing.assert_allclose(phi, direct.potential(x, x, s), rtol=1e-13)
    assert direct.rel_l2(g, direct.gradient(x, x, s)) < 1e-13


def test_error_falls_with_expansion_order():
    x, s = _small(2000)
    t = tree.Tree(x, 2, (0.5, 0.5, 0.5), 0.5)
    ref = direct.potential(x, x, s)
    errs = [direct.rel_l2(fmm.evaluate(t, operators.Operators(p, eps_pinv=1e-10), s, gradient=False)[0], ref)
            for p in (3, 4, 5, 6, 7)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[0] < 1e-3 and errs[-1] < 1e-7


@pytest.fixture(scope="module")
def config1():
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    xf, sf = workloads.make(w)
    x, s = xf.astype(np.float64), sf.astype(np.float64)
    c, r = w.cube
    t = tree.Tree(x, w.depth, c, r)
    ops = operators.Operators(w.p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
    return x, s, t, ops


def test_config1_against_direct_sum(config1):
    # 20,000 points uniform in the unit cube, depth 3, p = 6: compared with eq. (1) on 2,000
    # sampled targets (the full direct sum is the same formula on more rows).
    x, s, t, ops = config1
    phi, g = fmm.evaluate(t, ops, s)
    idx = workloads.sample_indices(len(x), 2000, 4001)
    assert direct.rel_l2(phi[idx], direct.potential(x[idx], x, s)) < 1e-6
    assert direct.rel_l2(g[idx], direct.gradient(x[idx], x, s)) < 1e-4


def test_linearity_in_charges(config1):
    # Every step is linear in s.  The truncated pseudo-inverses keep condition numbers up to
    # 1/eps_pinv = 1e7, so FP64 rounding is amplified to ~1e-11; the bound is 1e-10.
    x, s, t, ops = config1
    rng = np.random.default_rng(9)
    s2 = rng.standard_normal(len(x))
    a, b = 0.75, -2.5
    p1, g1 = fmm.evaluate(t, ops, s)
    p2, g2 = fmm.evaluate(t, ops, s2)
    p12, g12 = fmm.evaluate(t, ops, a * s + b * s2)
    assert direct.rel_l2(p12, a * p1 + b * p2) < 1e-10
    assert direct.rel_l2(g12, a * g1 + b * g2) < 1e-10
    # multiple right-hand sides at once give the columns separately
    pm, gm = fmm.evaluate(t, ops, np.stack([s, s2], axis=1))
    assert direct.rel_l2(pm[:, 1], p2) < 1e-10 and direct.rel_l2(gm[:, 0], g1) < 1e-10


def test_homogeneity_and_translation():
    x, s = _small(3000, 5)
    ops = operators.Operators(5)
    p0, g0 = fmm.evaluate(tree.Tree(x, 3, (0.5, 0.5, 0.5), 0.5), ops, s)
    # scaling coordinates and cube by 2 (exact in binary) divides phi by 2 and grad by 4
    p2, g2 = fmm.evaluate(tree.Tree(2.0 * x, 3, (1.0, 1.0, 1.0), 1.0), ops, s)
    assert direct.rel_l2(2.0 * p2, p0) < 1e-12 and direct.rel_l2(4.0 * g2, g0) < 1e-11
    # shifting points and cube leaves the result unchanged (up to rounding of the absolute
    # surface coordinates, amplified by the pseudo-inverses as in the linearity test)
    shift = np.array([0.25, -0.5, 1.0])
    p3, g3 = fmm.evaluate(tree.Tree(x + shift, 3, 0.5 + shift, 0.5), ops, s)
    assert direct.rel_l2(p3, p0) < 1e-9 and direct.rel_l2(g3, g0) < 1e-9


def test_compressed_matches_plain():
    x, s = _small(3000, 6)
    t = tree.Tree(x, 3, (0.5, 0.5, 0.5), 0.5)
    pp, gp = fmm.evaluate(t, operators.Operators(6, m2l="plain"), s)
    pc, gc = fmm.evaluate(t, operators.Operators(6, m2l="compressed", eps_svd=1e-7), s)
    assert direct.rel_l2(pc, pp) < 1e-8 and direct.rel_l2(gc, gp) < 1e-7


def test_gradient_is_derivative_of_represented_field():
    # Inside a leaf the FMM potential is the D2T field plus the U-list sum; its central
    # difference at a target equals the FMM gradient there (the self term 1/h cancels).
    x, s = _small(2000, 12)
    t = tree.Tree(x, 2, (0.5, 0.5, 0.5), 0.5)
    ops = operators.Operators(6)
    st = fmm.evaluate(t, ops, s, return_state=True)
    h = 1e-6
    for i in (0, 17, 999):
        leaf = tuple(int(v) for v in t.leaf_index[i])
        fd = [(fmm.local_field(t, ops, s, st, leaf, x[i:i + 1] + h * e)[0]
               - fmm.local_field(t, ops, s, st, leaf, x[i:i + 1] - h * e)[0]) / (2 * h) for e in np.eye(3)]
        np.testing.assert_allclose(st.grad[i], fd, rtol=2e-6, atol=1e-6 * np.abs(st.grad[i]).max())
        # and the represented potential at the target itself is the FMM output
        assert abs(fmm.local_field(t, ops, s, st, leaf, x[i:i + 1])[0] - st.phi[i]) < 1e-12 * abs(st.phi[i])


def test_sampled_evaluation_equals_full(config1):
    x, s, t, ops = config1
    full, gfull = fmm.evaluate(t, ops, s)
    leaves = [(0, 0, 0), (3, 4, 5), (7, 7, 7)]
    part, gpart = fmm.evaluate(t, ops, s, target_leaves=leaves)
    idx = np.concatenate([t.leaf_points[b] for b in leaves])
    np.testing.assert_array_equal(part[idx], full[idx])
    np.testing.assert_array_equal(gpart[idx], gfull[idx])
    assert np.isnan(part).sum() == len(x) - len(idx)
