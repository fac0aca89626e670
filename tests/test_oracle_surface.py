"""Pins of the oracle's kiFMM surfaces: point counts (Sections 4 and 5) and geometry."""

import numpy as np

from oracle import surface


def _golden(golden_dir):
    vals = {}
    with open(f"{golden_dir}/paper_values.txt") as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                name, value = line.split()[:2]
                vals[name] = int(value)
    return vals


def test_paper_surface_count_p3(golden_dir):
    g = _golden(golden_dir)
    assert len(surface.reference_surface(3)) == g["surface_points_p3"]
    assert 4 * len(surface.reference_surface(3)) == g["surface_bytes_p3_fp32"]


def test_surface_count_formula():
    for p in range(2, 11):
        s = surface.reference_surface(p)
        assert len(s) == surface.n_points(p) == 6 * (p - 1) ** 2 + 2
        # p^3 grid minus its (p-2)^3 interior, computed independently
        assert len(s) == p ** 3 - max(p - 2, 0) ** 3
    assert [surface.n_points(p) for p in (6, 7, 8)] == [152, 218, 296]


def test_surface_geometry():
    for p in (3, 6, 8):
        s = surface.reference_surface(p)
        np.testing.assert_array_equal(np.max(np.abs(s), axis=1), 1.0)
        assert len({tuple(v) for v in s}) == len(s)
        # symmetric under x -> -x
        assert {tuple(v) for v in s} == {tuple(-v) for v in s}
        # grid spacing 2/(p-1)
        steps = np.unique(np.round((s + 1.0) * (p - 1) / 2.0, 12))
        np.testing.assert_allclose(steps, np.arange(p))
    b = surface.box_surface(6, (1.0, 2.0, 3.0), 0.25, 2.95)
    np.testing.assert_allclose(np.max(np.abs(b - [1.0, 2.0, 3.0]), axis=1), 0.25 * 2.95)
