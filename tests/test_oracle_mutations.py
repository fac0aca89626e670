"""Plausible mistakes planted in the oracle must be caught by its pins.

Each case patches one piece of the oracle (on the CPU) and checks that the
direct-sum comparison, which pins the oracle, then fails by a wide margin.
"""

import numpy as np
import pytest

from oracle import direct, fmm, kernel, operators, tree


@pytest.fixture(scope="module")
def problem():
    rng = np.random.default_rng(31)
    x = rng.random((2000, 3))
    s = rng.random(2000)
    return x, s, direct.potential(x, x, s), direct.gradient(x, x, s)


def _errors(problem):
    x, s, ref, gref = problem
    t = tree.Tree(x, 3, (0.5, 0.5, 0.5), 0.5)
    phi, g = fmm.evaluate(t, operators.Operators(5), s)
    return direct.rel_l2(phi, ref), direct.rel_l2(g, gref)


def test_unmutated_oracle_passes(problem):
    e, eg = _errors(problem)
    assert e < 1e-5 and eg < 1e-3


MUTATIONS = {
    "v_list_drops_one": (tree.Tree, "v_list",
                         lambda orig: (lambda self, l, b: orig(self, l, b)[:-1])),
    "u_list_without_self": (tree.Tree, "u_list",
                            lambda orig: (lambda self, b: [a for a in orig(self, b) if a != b])),
    "m2m_transposed": (operators.Operators, "m2m_check",
                       lambda orig: (lambda self, r, o: orig(self, r, o).T)),
    "l2l_skipped": (operators.Operators, "l2l_check",
                    lambda orig: (lambda self, r, o: 0.0 * orig(self, r, o))),
    "m2l_wrong_sign_offset": (operators.Operators, "m2l_kernel",
                              lambda orig: (lambda self, r, t: orig(self, r, tuple(-v for v in t)))),
    "child_octant_bits_swapped": (operators, "child_offset",
                                  lambda orig: (lambda o, r: orig(((o & 1) << 1) | ((o >> 1) & 1) | (o & 4), r))),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(problem, monkeypatch, name):
    owner, attr, make = MUTATIONS[name]
    monkeypatch.setattr(owner, attr, make(getattr(owner, attr)))
    e, eg = _errors(problem)
    assert max(e / 1e-5, eg / 1e-3) > 10.0, (name, e, eg)


def test_gradient_sign_mutation_is_caught(monkeypatch):
    orig = kernel.gradient_matrix
    monkeypatch.setattr(kernel, "gradient_matrix", lambda x, y: -orig(x, y))
    rng = np.random.default_rng(4)
    src = rng.random((20, 3))
    s = rng.standard_normal(20)
    x = np.array([[0.3, 1.7, -0.4]])
    g = direct.gradient(x, src, s)[0]
    h = 1e-5
    fd = np.array([(direct.potential(x + h * e, src, s)[0] - direct.potential(x - h * e, src, s)[0]) / (2 * h)
                   for e in np.eye(3)])
    assert np.linalg.norm(g - fd) > 0.5 * np.linalg.norm(fd)
