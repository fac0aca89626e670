"""Pins of the oracle's kernel and direct sum (eq. (1)-(2)) against closed forms."""

import itertools
import math

import numpy as np
import pytest

from oracle import direct, kernel



def test_kernel_values_and_coincident_points():
    x = np.zeros((1, 3))
    y = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    k = kernel.potential_matrix(x, y)
    assert k[0, 0] == 0.2          # |(3,4,0)| = 5
    assert k[0, 1] == 0.0          # coincident pair contributes nothing
    assert k[0, 2] == 1.0 / 3.0    # |(1,2,2)| = 3


def test_gradient_closed_form():
    g = kernel.gradient_matrix(np.array([[3.0, 4.0, 0.0], [1.0, 1.0, 1.0]]),
                               np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]))
    np.testing.assert_allclose(g[0, 0], [-3.0 / 125.0, -4.0 / 125.0, 0.0], rtol=1e-15)
    np.testing.assert_array_equal(g[1, 1], [0.0, 0.0, 0.0])


def _icosahedron(a):
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1, s2 in itertools.product((-1.0, 1.0), repeat=2):
        v += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    v = np.array(v)
    return a * v / np.linalg.norm(v, axis=1, keepdims=True)


def test_icosahedron_far_field_is_monopole():
    # The 12 icosahedron vertices form a spherical 5-design, so multipole moments of
    # degree 1..5 vanish: at distance R = 10a the potential of 12 unit charges is 12/R
    # up to sum_{l>=6} (a/R)^l <= 1.2e-6 relative, and the field is radial, 12/R^2.
    a = 0.1
    src = _icosahedron(a)
    rng = np.random.default_rng(7)
    dirs = rng.standard_normal((16, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    R = 10.0 * a
    tgt = R * dirs
    phi = direct.potential(tgt, src, np.ones(12))
    np.testing.assert_allclose(phi, 12.0 / R, rtol=1.2e-6)
    grad = direct.gradient(tgt, src, np.ones(12))
    np.testing.assert_allclose(grad, -12.0 * tgt / R ** 3, rtol=0, atol=1e-5 * 12.0 / R ** 2)


def test_pair_energy_brute_force():
    # sum_i s_i phi_i counts every pair twice: 2 sum_{i<j} s_i s_j / r_ij (pure-Python loop).
    rng = np.random.default_rng(3)
    x = rng.random((9, 3))
    s = rng.standard_normal(9)
    e = 0.0
    for i in range(9):
        for j in range(i + 1, 9):
            d = math.sqrt(sum((x[i][c] - x[j][c]) ** 2 for c in range(3)))
            e += s[i] * s[j] / d
    phi = direct.potential(x, x, s)
    assert abs(float(s @ phi) - 2.0 * e) <= 1e-13 * abs(2.0 * e)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    src = rng.random((20, 3))
    s = rng.standard_normal(20)
    x = np.array([[0.3, 1.7, -0.4]])
    g = direct.gradient(x, src, s)[0]
    h = 1e-5
    fd = [(direct.potential(x + h * e, src, s)[0] - direct.potential(x - h * e, src, s)[0]) / (2 * h)
          for e in np.eye(3)]
    np.testing.assert_allclose(g, fd, rtol=1e-8)
