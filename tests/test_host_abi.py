"""CPU tests of the C-ABI library: exports, tree build and operator precompute against
the oracle, and error paths.  No device work is done (no GPU needed)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import operators as oops
from oracle import surface as osurf
from oracle import tree as otree
from paper_2604_19243_amd import kifmm, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return kifmm.library()


def test_library_exports_every_declared_symbol(lib):
    header = open(os.path.join(ROOT, "include", "kifmm_mi355x.h")).read()
    names = set(re.findall(r"\b(kifmm_[a-z_0-9]+)\s*\(", header))
    assert len(names) >= 18
    for name in sorted(names):
        assert hasattr(lib, name), name
    assert kifmm.kifmm_abi_version() == 3


@pytest.mark.parametrize("dist,depth,n", [("cube", 3, 20_000), ("cube", 5, 50_000), ("sphere", 4, 30_000),
                                          ("cube", 0, 100), ("cube", 1, 500)])
def test_tree_matches_oracle(dist, depth, n):
    x = workloads.points(dist, n, 77)
    cube = (0.5, 0.5, 0.5, 0.5) if dist == "cube" else (0.0, 0.0, 0.0, 1.0)
    t = kifmm.kifmm_tree_build_host(x, depth, cube)
    try:
        ref = otree.Tree(x.astype(np.float64), depth, cube[:3], cube[3])
        np.testing.assert_array_equal(kifmm.kifmm_tree_get_leaf_coords(t, n), ref.leaf_index)
        np.testing.assert_array_equal(kifmm.kifmm_tree_get_order(t, n), ref.order)
        info = kifmm.kifmm_tree_stats_get(t)
        assert info["nonempty_boxes"] == [len(b) for b in ref.boxes]
        assert info["max_leaf"] == max(len(v) for v in ref.leaf_points.values())
    finally:
        kifmm.kifmm_tree_destroy(t)


def test_tree_auto_cube_and_boundary_points():
    rng = np.random.default_rng(5)
    x = (rng.random((3000, 3)) * [2.0, 1.0, 0.5] - 0.3).astype(np.float32)
    x[0] = x.min(axis=0)
    x[1] = x.max(axis=0)
    t = kifmm.kifmm_tree_build_host(x, 4, None)
    try:
        ref = otree.Tree(x.astype(np.float64), 4)
        info = kifmm.kifmm_tree_stats_get(t)
        assert info["half_width"] == ref.half_width
        assert info["center"] == tuple(ref.center)
        np.testing.assert_array_equal(kifmm.kifmm_tree_get_leaf_coords(t, 3000), ref.leaf_index)
    finally:
        kifmm.kifmm_tree_destroy(t)


@pytest.fixture(scope="module", params=[(6, 1e-6), (5, 1e-7)])
def ops_pair(request):
    p, eps_svd = request.param
    h = kifmm.kifmm_ops_precompute(p, eps_pinv=1e-7, eps_svd=eps_svd)
    ref = oops.Operators(p, eps_pinv=1e-7, m2l="compressed", eps_svd=eps_svd)
    yield p, h, ref
    kifmm.kifmm_ops_destroy(h)


def test_ops_info_and_surface(ops_pair):
    p, h, ref = ops_pair
    info = kifmm.kifmm_ops_get_info(h)
    n = osurf.n_points(p)
    assert info["n_surface"] == n and info["n_m2l_offsets"] == 316
    uk = ref.compression(1.0)[0]
    assert info["rank_m2l"] == uk.shape[1]
    np.testing.assert_array_equal(kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_SURFACE, 0, (n, 3)), osurf.reference_surface(p))
    if p == 6:
        assert info["rank_m2l"] == 116


def test_check_to_equivalent_matches_oracle(ops_pair):
    p, h, ref = ops_pair
    n = osurf.n_points(p)
    for which, mine in ((kifmm.KIFMM_OP_UC2E, ref.uc2e(1.0)), (kifmm.KIFMM_OP_DC2E, ref.dc2e(1.0))):
        got = kifmm.kifmm_ops_get_matrix(h, which, 0, (n, n))
        # pinv of a matrix whose kept condition number is <= 1e7: agreement ~1e-16 * 1e7
        assert np.linalg.norm(got - mine) <= 1e-7 * np.linalg.norm(mine)


def test_translations_match_oracle(ops_pair):
    p, h, ref = ops_pair
    n = osurf.n_points(p)
    for oc in (0, 3, 7):
        m2m = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2M, oc, (n, n))
        want = ref.uc2e(2.0) @ ref.m2m_check(1.0, oc)
        assert np.linalg.norm(m2m - want) <= 1e-7 * np.linalg.norm(want)
        l2l = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_L2L, oc, (n, n))
        want = ref.dc2e(1.0) @ ref.l2l_check(1.0, oc)
        assert np.linalg.norm(l2l - want) <= 1e-7 * np.linalg.norm(want)


def test_compressed_m2l_matches_oracle(ops_pair):
    # Bases are not unique; compare the approximate operators U_k C_t V_k^T and the folded
    # post C_t V_k^T = DC2E U_k C_t V_k^T.
    p, h, ref = ops_pair
    n = osurf.n_points(p)
    k = kifmm.kifmm_ops_get_info(h)["rank_m2l"]
    U = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2L_U, 0, (n, k))
    V = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2L_V, 0, (n, k))
    post = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2L_POST, 0, (n, k))
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    ruk, rvk, rcores, _ = ref.compression(1.0)
    offs = oops.v_list_offsets()
    for idx in (0, 57, 150, 315):
        t = tuple(int(v) for v in kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2L_OFFSET, idx, (3,)))
        assert t == offs[idx]
        C = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2L_CORE, idx, (k, k))
        mine = U @ C @ V.T
        want = ruk @ rcores[t] @ rvk.T
        assert np.linalg.norm(mine - want) <= 1e-10 * np.linalg.norm(want)
        mine_post = post @ C @ V.T
        want_post = ref.dc2e(1.0) @ want
        assert np.linalg.norm(mine_post - want_post) <= 1e-7 * np.linalg.norm(want_post)


def _status(fn, *args):
    with pytest.raises(kifmm.KifmmError) as e:
        fn(*args)
    return e.value.status


def test_error_paths(lib):
    x = workloads.points("cube", 100, 1)
    assert _status(kifmm.kifmm_tree_build_host, x, -1) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_tree_build_host, x, 11) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_tree_build_host, x[:0], 2) == kifmm.KIFMM_E_INVALID
    bad = x.copy()
    bad[3, 1] = np.nan
    assert _status(kifmm.kifmm_tree_build_host, bad, 2) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_tree_build_host, x, 2, (0.5, 0.5, 0.5, 0.0)) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_tree_build_host, x, 2, (0.5, math.inf, 0.5, 1.0)) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_ops_precompute, 1) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_ops_precompute, 13) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_ops_precompute, 4, 1.05, 2.95, 0.0) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_ops_precompute, 4, 1.05, 2.95, 1e-7, 2.0) == kifmm.KIFMM_E_INVALID
    assert _status(kifmm.kifmm_ops_precompute, 4, 1.05, 2.95, 1e-7, -1000.0) == kifmm.KIFMM_E_INVALID  # rank > n
    assert _status(kifmm.kifmm_ops_precompute, 4, 1.05, 2.95, 1e-7, -2.5) == kifmm.KIFMM_E_INVALID    # not an integer
    # surface radii: 1 < alpha_inner < alpha_outer, alpha_inner + alpha_outer <= 4
    for ai, ao in ((1.0, 2.95), (0.9, 2.0), (2.0, 1.5), (1.5, 2.6), (1.05, math.nan)):
        assert _status(kifmm.kifmm_ops_precompute, 4, ai, ao) == kifmm.KIFMM_E_INVALID, (ai, ao)
    # null handles and pointers
    out = ctypes.c_void_p()
    assert lib.kifmm_tree_build_host(None, 10, 2, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
    assert lib.kifmm_tree_build(None, 10, 2, None, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
    assert lib.kifmm_tree_stats_get(None, None) == kifmm.KIFMM_E_INVALID
    assert lib.kifmm_evaluate(None, None, None, None, None) == kifmm.KIFMM_E_INVALID
    assert b"null" in lib.kifmm_last_error()
    assert lib.kifmm_plan_destroy(None) == kifmm.KIFMM_E_INVALID
    t = kifmm.kifmm_tree_build_host(x, 2, (0.5, 0.5, 0.5, 0.5))
    o = kifmm.kifmm_ops_precompute(3)
    try:
        assert lib.kifmm_ops_get_matrix(o, 99, 0, None, 0) == kifmm.KIFMM_E_INVALID
        buf = np.zeros(4)
        assert lib.kifmm_ops_get_matrix(o, kifmm.KIFMM_OP_SURFACE, 0, buf.ctypes.data, 4) == kifmm.KIFMM_E_INVALID
        assert b"capacity" in lib.kifmm_last_error()
        assert lib.kifmm_plan_create(t, o, 1, 0, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
        assert lib.kifmm_plan_create(t, o, 3, 1, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
        assert lib.kifmm_plan_create(t, o, 4, 3, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
        for pair in ((kifmm.KIFMM_UPPER_STREAM, kifmm.KIFMM_NO_UPPER_STREAM),
                     (kifmm.KIFMM_LEAF_THREADS_256, kifmm.KIFMM_LEAF_THREADS_320),
                     (kifmm.KIFMM_LEAF_QUEUE, kifmm.KIFMM_LEAF_BLOCKS),
                     (kifmm.KIFMM_M2L_BF16X3, kifmm.KIFMM_M2L_BF16X6),
                     (kifmm.KIFMM_M2L_BLOCKED, kifmm.KIFMM_M2L_GATHER)):
            both = kifmm.KIFMM_POTENTIAL | pair[0] | pair[1]
            assert lib.kifmm_plan_create(t, o, 1, both, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID, pair
        assert lib.kifmm_plan_create(t, o, 1, 1 | 32768, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
        assert lib.kifmm_plan_create(t, o, 4, 1 | kifmm.KIFMM_LEAF_QUEUE, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
    finally:
        kifmm.kifmm_ops_destroy(o)
        kifmm.kifmm_tree_destroy(t)


def test_plan_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    x = workloads.points("cube", 100, 1)
    t = kifmm.kifmm_tree_build_host(x, 2, (0.5, 0.5, 0.5, 0.5))
    o = kifmm.kifmm_ops_precompute(3)
    try:
        with pytest.raises(kifmm.KifmmError) as e:
            kifmm.kifmm_plan_create(t, o)
        assert e.value.status in (kifmm.KIFMM_E_DEVICE, kifmm.KIFMM_E_INVALID)
    finally:
        kifmm.kifmm_ops_destroy(o)
        kifmm.kifmm_tree_destroy(t)


def test_binding_constants_match_the_header():
    # every #define KIFMM_* and every KIFMM_* = value in an enum of the header has the
    # same value in the binding
    header = open(os.path.join(ROOT, "include", "kifmm_mi355x.h")).read()
    found = dict(re.findall(r"#define\s+(KIFMM_[A-Z0-9_]+)\s+(-?\d+)u?\b", header))
    found.update(re.findall(r"\b(KIFMM_[A-Z0-9_]+)\s*=\s*(-?\d+)", header))
    assert len(found) >= 20
    for name, value in found.items():
        if hasattr(kifmm, name):
            assert getattr(kifmm, name) == int(value), name
    # the binding's stage names in the header's stage order, and the library's ABI version
    for i, stage in enumerate(kifmm.STAGES):
        assert int(found["KIFMM_STAGE_" + stage.upper()]) == i, stage
    assert int(found["KIFMM_N_STAGES"]) == len(kifmm.STAGES)
    assert int(found["KIFMM_ABI_VERSION"]) == kifmm.kifmm_abi_version()
    for name in ("KIFMM_POTENTIAL", "KIFMM_GRADIENT", "KIFMM_SERIAL", "KIFMM_M2L_BF16X3", "KIFMM_M2L_BF16X6",
                 "KIFMM_VJP", "KIFMM_M2L_BLOCKED", "KIFMM_M2L_GATHER", "KIFMM_UPPER_STREAM", "KIFMM_NO_UPPER_STREAM",
                 "KIFMM_LEAF_THREADS_256", "KIFMM_LEAF_THREADS_320", "KIFMM_LEAF_QUEUE", "KIFMM_LEAF_BLOCKS",
                 "KIFMM_NO_AUTOTUNE",
                 "KIFMM_N_STATS", "KIFMM_E_INVALID", "KIFMM_E_DEVICE", "KIFMM_E_STATE", "KIFMM_E_NOMEM"):
        assert name in found and hasattr(kifmm, name), name
    # the interface's flag values: potentials 1, gradients 2, split-bfloat16 M2L 4
    assert (kifmm.KIFMM_POT, kifmm.KIFMM_GRAD, kifmm.KIFMM_M2L_BF16X3) == (1, 2, 4)
    assert len(kifmm.STATS_KEYS) == kifmm.KIFMM_N_STATS


def test_parent_target_counts_of_the_1m_workload():
    # The leaf kernels take one parent (8 sibling leaves) per workgroup. On the 1M-point, depth-5
    # workload a parent holds 244 targets on average: about a fifth exceed 256 (a second pass with
    # 256 threads) and none exceeds 320 (one pass with 320 threads).
    w = workloads.WORKLOADS["cube1m_p6_d5"]
    x, _ = workloads.make(w)
    t = kifmm.kifmm_tree_build_host(x, w.depth, w.cube[0] + (w.cube[1],))
    try:
        ijk = np.asarray(kifmm.kifmm_tree_get_leaf_coords(t, len(x))).astype(np.int64)
    finally:
        kifmm.kifmm_tree_destroy(t)
    side = 1 << (w.depth - 1)
    par = ijk >> 1
    counts = np.bincount((par[:, 0] * side + par[:, 1]) * side + par[:, 2], minlength=side ** 3)
    assert counts.sum() == w.n and abs(counts.mean() - w.n / side ** 3) < 1e-9
    assert 0.15 < (counts > 256).mean() < 0.30
    assert counts.max() <= 320


def test_destroyed_and_unknown_handles_give_state_errors(lib):
    # Handles are registry identifiers that are never reused: a destroyed handle, a second
    # destroy, a value the library never returned, and a handle of another kind all give
    # KIFMM_E_STATE without touching freed memory.
    x = workloads.points("cube", 200, 3)
    t = kifmm.kifmm_tree_build_host(x, 2, (0.5, 0.5, 0.5, 0.5))
    o = kifmm.kifmm_ops_precompute(3)
    stats = kifmm.TreeStats()
    assert lib.kifmm_tree_stats_get(t, ctypes.byref(stats)) == kifmm.KIFMM_OK
    assert lib.kifmm_tree_stats_get(o, ctypes.byref(stats)) == kifmm.KIFMM_E_STATE       # an ops handle
    assert lib.kifmm_ops_destroy(t) == kifmm.KIFMM_E_STATE                               # a tree handle
    kifmm.kifmm_tree_destroy(t)
    assert lib.kifmm_tree_stats_get(t, ctypes.byref(stats)) == kifmm.KIFMM_E_STATE
    assert b"destroyed" in lib.kifmm_last_error()
    assert lib.kifmm_tree_destroy(t) == kifmm.KIFMM_E_STATE
    assert lib.kifmm_tree_stats_get(ctypes.c_void_p(0x12345678), ctypes.byref(stats)) == kifmm.KIFMM_E_STATE
    out = ctypes.c_void_p()
    assert lib.kifmm_plan_create(t, o, 1, 1, None, ctypes.byref(out)) == kifmm.KIFMM_E_STATE
    assert lib.kifmm_evaluate(ctypes.c_void_p(0x7777), None, None, None, None) == kifmm.KIFMM_E_STATE
    kifmm.kifmm_ops_destroy(o)
    assert lib.kifmm_ops_destroy(o) == kifmm.KIFMM_E_STATE
    # a new object never reuses an old handle value
    t2 = kifmm.kifmm_tree_build_host(x, 2, (0.5, 0.5, 0.5, 0.5))
    assert t2.value != t.value
    kifmm.kifmm_tree_destroy(t2)


def test_workspace_bytes_and_device_memory_limit():
    # The plan's device bytes are known from host work alone; above the process-wide limit
    # plan creation fails with KIFMM_E_NOMEM before any device call (here, on a machine
    # without a GPU, the same call otherwise fails at the first device call).
    import torch
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    x, _ = workloads.make(w)
    t = kifmm.kifmm_tree_build_host(x, w.depth, w.cube[0] + (w.cube[1],))
    o = kifmm.kifmm_ops_precompute(w.p)
    try:
        flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT
        b = kifmm.kifmm_plan_workspace_bytes(t, o, 1, flags)
        # at least the sorted points, the per-box densities u, d of levels 2..3 and the 316 cores
        n, k = 152, kifmm.kifmm_ops_get_info(o)["rank_m2l"]
        assert b > 16 * w.n + 2 * 4 * n * (64 + 512) + 316 * 4 * k * k
        assert kifmm.kifmm_plan_workspace_bytes(t, o, 1, flags | kifmm.KIFMM_VJP) >= b + 2 * 12 * w.n
        assert kifmm.kifmm_plan_workspace_bytes(t, o, 4, kifmm.KIFMM_POTENTIAL) > b
        with pytest.raises(kifmm.KifmmError) as e:
            kifmm.kifmm_plan_workspace_bytes(t, o, 3, flags)
        assert e.value.status == kifmm.KIFMM_E_INVALID
        with pytest.raises(kifmm.KifmmError) as e:
            kifmm.kifmm_set_device_memory_limit(-1)
        assert e.value.status == kifmm.KIFMM_E_INVALID
        kifmm.kifmm_set_device_memory_limit(b - 1)
        try:
            with pytest.raises(kifmm.KifmmError) as e:
                kifmm.kifmm_plan_create(t, o, 1, flags)
            assert e.value.status == kifmm.KIFMM_E_NOMEM and "limit" in str(e.value)
        finally:
            kifmm.kifmm_set_device_memory_limit(0)
        if not torch.cuda.is_available():
            with pytest.raises(kifmm.KifmmError) as e:
                kifmm.kifmm_plan_create(t, o, 1, flags)
            assert e.value.status == kifmm.KIFMM_E_DEVICE
    finally:
        kifmm.kifmm_ops_destroy(o)
        kifmm.kifmm_tree_destroy(t)


def test_surface_radii_and_rank_arguments():
    # alpha_inner / alpha_outer reach every operator: the library's UC2E and U2U at
    # (1.2, 2.7) match the oracle's built at the same radii; a negative eps_svd gives
    # the rank (extended to the end of a singular-value cluster).
    p, ai, ao = 4, 1.2, 2.7
    h = kifmm.kifmm_ops_precompute(p, ai, ao, 1e-7, 1e-6)
    try:
        info = kifmm.kifmm_ops_get_info(h)
        assert (info["alpha_inner"], info["alpha_outer"]) == (ai, ao)
        ref = oops.Operators(p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6, alpha_inner=ai, alpha_outer=ao)
        n = osurf.n_points(p)
        got = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_UC2E, 0, (n, n))
        assert np.linalg.norm(got - ref.uc2e(1.0)) <= 1e-7 * np.linalg.norm(ref.uc2e(1.0))
        m2m = kifmm.kifmm_ops_get_matrix(h, kifmm.KIFMM_OP_M2M, 5, (n, n))
        want = ref.uc2e(2.0) @ ref.m2m_check(1.0, 5)
        assert np.linalg.norm(m2m - want) <= 1e-7 * np.linalg.norm(want)
        assert info["rank_m2l"] == ref.compression(1.0)[0].shape[1]
        default = oops.Operators(p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
        assert np.linalg.norm(ref.uc2e(1.0) - default.uc2e(1.0)) > 1e-3 * np.linalg.norm(default.uc2e(1.0))
    finally:
        kifmm.kifmm_ops_destroy(h)
    h = kifmm.kifmm_ops_precompute(6, eps_svd=-94.0)
    try:
        info = kifmm.kifmm_ops_get_info(h)
        assert info["rank_m2l"] == 94 and info["eps_svd"] == -94.0
    finally:
        kifmm.kifmm_ops_destroy(h)


def test_device_tree_build_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = kifmm.library()
    out = ctypes.c_void_p()
    assert lib.kifmm_tree_build(ctypes.c_void_p(4096), 10, 2, None, None, ctypes.byref(out)) == kifmm.KIFMM_E_DEVICE
    assert lib.kifmm_tree_build(ctypes.c_void_p(4096), 0, 2, None, None, ctypes.byref(out)) == kifmm.KIFMM_E_INVALID
