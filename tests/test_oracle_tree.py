"""Pins of the oracle's octree, Morton keys and U/V lists (Section 2.1, Table 1)."""

import itertools

import numpy as np

from oracle import operators, tree
from test_oracle_surface import _golden


def test_morton_examples():
    assert tree.morton_key(1, 0, 0, 3) == 1
    assert tree.morton_key(0, 1, 0, 3) == 2
    assert tree.morton_key(0, 0, 1, 3) == 4
    assert tree.morton_key(1, 1, 1, 3) == 7
    assert tree.morton_key(2, 0, 0, 3) == 8
    # ix=3 (011), iy=5 (101), iz=7 (111): triples (z,y,x) per bit 111, 101, 110 -> 7 + 5*8 + 6*64
    assert tree.morton_key(3, 5, 7, 3) == 7 + 40 + 384
    idx = np.array([[3, 5, 7], [1, 0, 0], [7, 7, 7]])
    np.testing.assert_array_equal(tree.morton_keys(idx, 3), [431, 1, 511])


def test_sorted_keys_are_preorder():
    # Parent key = child key >> 3, so sorting leaf keys groups every subtree contiguously.
    rng = np.random.default_rng(11)
    t = tree.Tree(rng.random((3000, 3)), 4, (0.5, 0.5, 0.5), 0.5)
    keys = t.keys[t.order]
    for shift in (3, 6, 9):
        anc = keys >> np.uint64(shift)
        change = np.flatnonzero(anc[1:] != anc[:-1])
        # each ancestor value appears in one contiguous run
        assert len(np.unique(anc)) == len(change) + 1
    # key of the box at level l equals morton_key of its coordinates at that level
    for pos in t.order[:50]:
        i = t.leaf_index[pos]
        for l in range(5):
            assert int(t.keys[pos]) >> (3 * (4 - l)) == tree.morton_key(*(i >> (4 - l)), l)


def test_leaf_assignment_faces():
    pts = np.array([[0.0, 0.0, 0.0],        # lower corner -> box 0
                    [1.0, 1.0, 1.0],        # top face -> clamped into the last box
                    [0.25, 0.5, 0.75],      # on interior faces -> the upper box (floor)
                    [0.2499999, 0.5, 0.7500001]])
    idx = tree.leaf_coordinates(pts, 2, (0.5, 0.5, 0.5), 0.5)
    np.testing.assert_array_equal(idx, [[0, 0, 0], [3, 3, 3], [1, 2, 3], [0, 2, 3]])


def test_stable_order_for_equal_keys():
    pts = np.array([[0.1, 0.1, 0.1], [0.9, 0.9, 0.9], [0.11, 0.1, 0.1], [0.12, 0.1, 0.1]])
    t = tree.Tree(pts, 1, (0.5, 0.5, 0.5), 0.5)
    np.testing.assert_array_equal(t.order, [0, 2, 3, 1])
    np.testing.assert_array_equal(t.leaf_points[(0, 0, 0)], [0, 2, 3])


def _full_tree(depth):
    m = 2 ** depth
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / m
    return tree.Tree(g, depth, (0.5, 0.5, 0.5), 0.5)


def test_list_sizes_and_paper_neighbour_counts(golden_dir):
    gold = _golden(golden_dir)
    t = _full_tree(3)
    interior = (3, 4, 3)
    assert len(t.colleagues(3, interior)) == gold["max_adjacent_boxes"]
    assert len(tree.Tree.children(interior)) == gold["children_per_box"]
    assert len(t.u_list(interior)) == 27
    for box in t.boxes[3]:
        assert len(t.u_list(box)) <= 27
        v = t.v_list(3, box)
        assert len(v) <= 189
        for a in v:
            assert max(abs(a[i] - box[i]) for i in range(3)) in (2, 3)
            # parents are colleagues
            pa, pb = tree.Tree.parent(a), tree.Tree.parent(box)
            assert max(abs(pa[i] - pb[i]) for i in range(3)) == 1
    assert len(t.v_list(3, interior)) == 189
    assert t.v_list(1, (0, 0, 0)) == []


def test_full_tree_pair_counts_closed_form():
    # Per axis, a box at level l (m = 2^l boxes) has b(i) adjacent positions (itself included)
    # and a(i) positions whose parent is within one of its parent; V = product(a) - product(b)
    # per box, hence (sum a)^3 - (sum b)^3 pairs, with sum b = 3m-2 and sum a = 6m-8.
    for depth in (2, 3, 4):
        t = _full_tree(depth)
        m = 2 ** depth
        for l in range(2, depth + 1):
            ml = 2 ** l
            v_pairs = sum(len(t.v_list(l, b)) for b in t.boxes[l])
            assert v_pairs == (6 * ml - 8) ** 3 - (3 * ml - 2) ** 3
        u_pairs = sum(len(t.u_list(b)) for b in t.boxes[depth])
        assert u_pairs == (3 * m - 2) ** 3
    assert (6 * 32 - 8) ** 3 - (3 * 32 - 2) ** 3 == 5_398_920


def test_v_offsets_closed_form():
    offs = operators.v_list_offsets()
    closed = [t for t in itertools.product(range(-3, 4), repeat=3) if max(map(abs, t)) in (2, 3)]
    assert sorted(offs) == sorted(closed)
    assert len(offs) == 7 ** 3 - 3 ** 3 == 316
    # per position among siblings, an interior box sees 189 of them
    t = _full_tree(3)
    for box in [(2, 2, 2), (3, 2, 2), (2, 3, 3), (3, 3, 3)]:
        assert len({(box[0] - a[0], box[1] - a[1], box[2] - a[2]) for a in t.v_list(3, box)}) == 189
