"""Pins of the oracle's kiFMM operators (Table 1) against identities that hold mathematically."""

import numpy as np
import pytest

from oracle import direct, kernel, operators


@pytest.fixture(scope="module")
def ops6():
    return operators.Operators(6, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-7)


def test_pinv_moore_penrose_when_untruncated():
    # p = 3: cond(K(UC,UE)) ~ 2e3, so nothing is truncated and the Moore-Penrose
    # conditions hold to rounding.
    ops = operators.Operators(3, eps_pinv=1e-10)
    for a in (kernel.potential_matrix(ops.upward_check(1.0), ops.upward_equivalent(1.0)),
              kernel.potential_matrix(ops.downward_check(1.0), ops.downward_equivalent(1.0))):
        x = operators.pinv(a, 1e-10)
        np.testing.assert_allclose(a @ x @ a, a, atol=1e-12 * np.abs(a).max())
        np.testing.assert_allclose(x @ a @ x, x, atol=1e-10 * np.abs(x).max())
        np.testing.assert_allclose(a @ x, (a @ x).T, atol=1e-11)
        np.testing.assert_allclose(x @ a, (x @ a).T, atol=1e-11)


def _sources_in_box(rng, center, r, m=40):
    return center + r * (2.0 * rng.random((m, 3)) - 1.0), rng.random(m)


def test_upward_density_reproduces_far_field(ops6):
    # u = pinv(K(UC,UE)) K(UC,y) s reproduces the sources' field outside the check surface.
    rng = np.random.default_rng(5)
    r = 0.125
    y, s = _sources_in_box(rng, np.zeros(3), r)
    u = ops6.uc2e(r) @ (kernel.potential_matrix(ops6.upward_check(r), y) @ s)
    far = 4.0 * r * np.array([[1.0, 0.3, -0.2], [0.1, -1.0, 0.5], [0.7, 0.7, 1.0]])
    approx = kernel.potential_matrix(far, ops6.upward_equivalent(r)) @ u
    exact = direct.potential(far, y, s)
    np.testing.assert_allclose(approx, exact, rtol=2e-5)


def test_downward_density_reproduces_near_field(ops6):
    # d = pinv(K(DC,DE)) f(DC) reproduces a far source's field inside the box.
    rng = np.random.default_rng(6)
    r = 0.125
    y, s = _sources_in_box(rng, np.array([5.0 * r, -4.0 * r, 4.0 * r]), r)
    d = ops6.dc2e(r) @ direct.potential(ops6.downward_check(r), y, s)
    x = r * (2.0 * rng.random((30, 3)) - 1.0)
    np.testing.assert_allclose(kernel.potential_matrix(x, ops6.downward_equivalent(r)) @ d,
                               direct.potential(x, y, s), rtol=2e-5)


def test_check_to_equivalent_scaling():
    # K is homogeneous of degree -1, so pinv(K) at radius 2r is twice that at radius r.
    ops = operators.Operators(6, eps_pinv=1e-7)
    np.testing.assert_allclose(ops.uc2e(0.5), 2.0 * ops.uc2e(0.25), rtol=0, atol=1e-7 * np.abs(ops.uc2e(0.5)).max())
    np.testing.assert_allclose(ops.dc2e(0.5), 2.0 * ops.dc2e(0.25), rtol=0, atol=1e-7 * np.abs(ops.dc2e(0.5)).max())


def test_m2m_then_far_field(ops6):
    # U2U: the parent's density reproduces the field of the children's densities far away.
    rng = np.random.default_rng(8)
    rc = 0.125
    check = np.zeros(ops6.n)
    ys, ss = [], []
    for oc in range(8):
        y, s = _sources_in_box(rng, operators.child_offset(oc, rc), rc, 10)
        u = ops6.uc2e(rc) @ (kernel.potential_matrix(ops6.upward_check(rc, operators.child_offset(oc, rc)), y) @ s)
        check += ops6.m2m_check(rc, oc) @ u
        ys.append(y)
        ss.append(s)
    up = ops6.uc2e(2 * rc) @ check
    far = 8.0 * rc * np.array([[1.0, 0.2, 0.1], [-0.5, 1.0, 0.4]])
    np.testing.assert_allclose(kernel.potential_matrix(far, ops6.upward_equivalent(2 * rc)) @ up,
                               direct.potential(far, np.vstack(ys), np.concatenate(ss)), rtol=5e-5)


def test_compression_error_bound(ops6):
    # ||K_t - U U^T K_t V V^T||_F <= ||(I-UU^T) K_fat||_F + ||K_tall (I-VV^T)||_F
    #                              = sqrt(sum_{i>k} sf_i^2) + sqrt(sum_{i>k} st_i^2).
    r = 0.25
    uk, vk, cores, (sf, st) = ops6.compression(r)
    k = uk.shape[1]
    bound = np.sqrt(np.sum(sf[k:] ** 2)) + np.sqrt(np.sum(st[k:] ** 2))
    worst = 0.0
    for t in [(2, 0, 0), (3, 3, 3), (-2, 1, -3), (0, -3, 2)]:
        kt = ops6.m2l_kernel(r, t)
        worst = max(worst, np.linalg.norm(kt - uk @ cores[t] @ vk.T))
    assert worst <= bound * (1 + 1e-6)
    assert worst <= 1e-6 * sf[0]
    np.testing.assert_allclose(uk.T @ uk, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(vk.T @ vk, np.eye(k), atol=1e-12)


def test_compression_rank_and_clusters(ops6):
    uk, _, _, (sf, st) = ops6.compression(0.25)
    k = uk.shape[1]
    assert k == 143      # eps_svd = 1e-7 at p = 6
    assert (sf[k - 1] - sf[k]) > 1e-8 * sf[k - 1]
    assert (st[k - 1] - st[k]) > 1e-8 * st[k - 1]
    # the stacked spectrum has exact multiplicities from the cube's symmetry
    gaps = (sf[:-1] - sf[1:]) / sf[:-1]
    assert np.sum(gaps < 1e-8) > 20
    # scale invariance of the rank rule: same rank at another level
    assert ops6.compression(0.125)[0].shape[1] == k
