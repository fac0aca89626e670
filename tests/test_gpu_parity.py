"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded inputs.

Tolerance: relative L2 <= 1e-6 for potentials and gradients of the plain FP32 path.
"""

import numpy as np
import pytest

from gpu_helpers import assert_parity, gpu_evaluate, leaf_groups, log, oracle_evaluate, rel_l2
from oracle import direct
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6
UNIT = (0.5, 0.5, 0.5, 0.5)


@pytest.mark.parametrize("depth,n", [(0, 700), (1, 3000), (1, 1)])
def test_shallow_tree_equals_direct_sum(depth, n):
    # depth <= 1: every leaf is in every U list, so the HIP path is the direct sum (P2P only).
    log(f"shallow depth={depth} n={n}")
    x = workloads.points("cube", n, 10 + depth)
    s = workloads.charges("uniform01", n, 20 + depth)
    phi, g, f = gpu_evaluate(x, s, depth, 4, UNIT)
    f.close()
    x64, s64 = x.astype(np.float64), s.astype(np.float64)
    ref = direct.potential(x64, x64, s64)
    gref = direct.gradient(x64, x64, s64)
    if n == 1:
        assert phi[0] == 0.0 and np.all(g[0] == 0.0)
        return
    assert rel_l2(phi, ref) < TOL
    assert rel_l2(g, gref) < TOL


@pytest.mark.parametrize("name,n,depth,p,dist,serial,rank", [
    ("cube20k_p6_d3", 20_000, 3, 6, "cube", False, 0),   # the FP64 validation workload, full size
    ("cube20k_p6_d3", 20_000, 3, 6, "cube", True, 0),    # same, every kernel on the caller's stream
    ("ragged", 7_777, 4, 5, "cube", False, 0),           # ragged leaves and tiles, many boundary boxes
    ("sphere", 30_000, 4, 6, "sphere", False, 0),        # strongly non-uniform: most boxes empty
    ("sparse_deep", 2_000, 5, 4, "cube", True, 0),       # ~0.06 points per leaf
    ("depth2", 5_000, 2, 5, "cube", False, 0),           # far field at level 2 only: no U2U, no D2D
    ("depth2_serial", 5_000, 2, 5, "cube", True, 0),
    # rank 94 (the p = 6 benchmark rank): k padded to 96, three 32-row blocks, 32-k slabs
    ("rank94", 40_000, 4, 6, "cube", False, 94),
    ("rank94_sphere", 30_000, 4, 6, "sphere", False, 94),
])
def test_parity_with_oracle(name, n, depth, p, dist, serial, rank):
    log(f"parity {name} n={n} depth={depth} p={p} serial={serial} rank={rank}")
    x = workloads.points(dist, n, 1001 if name.startswith("cube20k") else 500 + n)
    s = workloads.charges("uniform01", n, 2001 if name.startswith("cube20k") else 600 + n)
    cube = UNIT if dist == "cube" else (0.0, 0.0, 0.0, 1.0)
    phi, g, f = gpu_evaluate(x, s, depth, p, cube, serial=serial, rank=rank)
    k = kifmm.kifmm_ops_get_info(f.ops)["rank_m2l"]
    f.close()
    rphi, rg, t, ops = oracle_evaluate(x, s, depth, p, cube, rank=rank or None)
    assert ops.compression(1.0)[0].shape[1] == k
    groups = leaf_groups(t)
    assert_parity(f"phi (k={k})", phi, rphi, groups, TOL)
    assert_parity("grad", g, rg, groups, TOL)


def test_linearity_and_determinism():
    log("linearity/determinism")
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    x, s1 = workloads.make(w)
    s2 = workloads.charges("normal", len(x), 99)
    c = w.cube[0] + (w.cube[1],)
    p1, g1, f = gpu_evaluate(x, s1, w.depth, w.p, c)
    p1b, g1b, _ = gpu_evaluate(x, s1, w.depth, w.p, c, fmm_obj=f)
    np.testing.assert_array_equal(p1, p1b)   # no atomics: bitwise repeatable
    np.testing.assert_array_equal(g1, g1b)
    p2, g2, _ = gpu_evaluate(x, s2, w.depth, w.p, c, fmm_obj=f)
    s12 = (0.5 * s1.astype(np.float64) - 2.0 * s2.astype(np.float64)).astype(np.float32)
    p12, g12, _ = gpu_evaluate(x, s12, w.depth, w.p, c, fmm_obj=f)
    f.close()
    assert rel_l2(p12, 0.5 * p1 - 2.0 * p2) < 1e-5
    assert rel_l2(g12, 0.5 * g1 - 2.0 * g2) < 1e-5


def test_full_size_hot_path_sampled():
    # 1,000,000 points, depth 5, p = 6: the benchmarked workload in the benchmarked launch
    # configuration, checked against the oracle on the points of 24 sampled leaves; the
    # single-stream configuration must give the same numbers to FP32 summation order.
    w = workloads.WORKLOADS["cube1m_p6_d5"]
    log("full size cube1m_p6_d5")
    x, s = workloads.make(w)
    c = w.cube[0] + (w.cube[1],)
    phi, g, f = gpu_evaluate(x, s, w.depth, w.p, c, rank=w.m2l_rank)
    assert kifmm.kifmm_ops_get_info(f.ops)["rank_m2l"] == w.m2l_rank
    f.close()
    phi_s, g_s, f = gpu_evaluate(x, s, w.depth, w.p, c, rank=w.m2l_rank, serial=True)
    f.close()
    assert rel_l2(phi_s, phi) < 1e-7 and rel_l2(g_s, g) < 1e-7
    assert np.isfinite(phi).all() and np.isfinite(g).all()
    rng = np.random.default_rng(4002)
    m = 2 ** w.depth
    leaves = {tuple(int(v) for v in rng.integers(0, m, 3)) for _ in range(20)}
    leaves |= {(0, 0, 0), (m - 1, m - 1, m - 1), (0, m - 1, 5), (m // 2, 0, m - 1)}
    leaves = sorted(leaves)
    rphi, rg, t, _ = oracle_evaluate(x, s, w.depth, w.p, c, rank=w.m2l_rank, target_leaves=leaves)
    groups = leaf_groups(t, leaves)
    assert_parity("phi, sampled leaves", phi, rphi, groups, TOL)
    assert_parity("grad, sampled leaves", g, rg, groups, TOL)


def test_stream_and_outputs_subset():
    import torch
    log("stream/outputs")
    x = workloads.points("cube", 5000, 3)
    s = workloads.charges("uniform01", 5000, 4)
    f = kifmm.FMM(x, 3, 4, cube=UNIT)
    dev = torch.device("cuda:0")
    st = torch.cuda.Stream()
    sd = torch.from_numpy(s).to(dev)
    pot = torch.zeros(5000, device=dev)
    grad = torch.zeros(5000, 3, device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        f.evaluate(sd, pot, grad, stream=st.cuda_stream)
        pot_only = torch.zeros(5000, device=dev)
        f.evaluate(sd, pot_only, None, stream=st.cuda_stream)
    st.synchronize()
    np.testing.assert_array_equal(pot.cpu().numpy(), pot_only.cpu().numpy())
    with pytest.raises(kifmm.KifmmError):
        f.evaluate(sd, None, None)
    f.close()


@pytest.mark.parametrize("p,n,depth", [
    (2, 3_000, 3),    # n = 8 surface points, k = 8: one 8-k chunk, one 32-row block
    (3, 5_000, 3),    # k = 26 -> 32 (zero-padded k)
    (7, 8_000, 3),    # k = 122 -> 128: four 40-k slabs, the last one 8 wide
    (8, 8_000, 3),    # n = 296, k = 124 -> 128
])
def test_expansion_orders(p, n, depth):
    log(f"order p={p} n={n} depth={depth}")
    x = workloads.points("cube", n, 700 + p)
    s = workloads.charges("uniform11", n, 800 + p)
    phi, g, f = gpu_evaluate(x, s, depth, p, UNIT)
    k = kifmm.kifmm_ops_get_info(f.ops)["rank_m2l"]
    f.close()
    rphi, rg, t, ops = oracle_evaluate(x, s, depth, p, UNIT)
    assert ops.compression(1.0)[0].shape[1] == k
    assert_parity(f"phi (k={k})", phi, rphi, leaf_groups(t), TOL)
    assert_parity("grad", g, rg, leaf_groups(t), TOL)


def test_orders_above_8_need_a_shallow_tree():
    # p = 9 (386 surface points): the leaf kernels hold at most 304, so a tree with a far
    # field is refused with KIFMM_E_INVALID; at depth 1 (the direct sum) the order is unused.
    log("order p=9")
    x = workloads.points("cube", 3_000, 709)
    s = workloads.charges("uniform11", 3_000, 809)
    ops = kifmm.kifmm_ops_precompute(9)
    try:
        for depth, ok in ((3, False), (1, True)):
            tree = kifmm.kifmm_tree_build_host(x, depth, UNIT)
            try:
                if ok:
                    plan = kifmm.kifmm_plan_create(tree, ops, 1, kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT)
                    kifmm.kifmm_plan_destroy(plan)
                else:
                    with pytest.raises(kifmm.KifmmError) as e:
                        kifmm.kifmm_plan_create(tree, ops, 1, kifmm.KIFMM_POTENTIAL)
                    assert e.value.status == kifmm.KIFMM_E_INVALID and "p <= 8" in str(e.value)
            finally:
                kifmm.kifmm_tree_destroy(tree)
    finally:
        kifmm.kifmm_ops_destroy(ops)


@pytest.mark.parametrize("depth", [8, 10])
def test_deep_sparse_trees(depth):
    # Maximum depth: almost every leaf holds one point and most boxes are empty.
    log(f"deep depth={depth}")
    n = 600
    x = workloads.points("sphere", n, 900 + depth)
    s = workloads.charges("uniform01", n, 901 + depth)
    phi, g, f = gpu_evaluate(x, s, depth, 4, (0.0, 0.0, 0.0, 1.0))
    f.close()
    rphi, rg, t, _ = oracle_evaluate(x, s, depth, 4, (0.0, 0.0, 0.0, 1.0))
    assert_parity("phi", phi, rphi, leaf_groups(t), TOL)
    assert_parity("grad", g, rg, leaf_groups(t), TOL)


def test_gradient_only_and_auto_cube():
    import torch
    log("gradient only, automatic cube")
    n = 6000
    x = (workloads.points("cube", n, 31) * np.float32(3.0) - np.float32(1.0)).astype(np.float32)
    s = workloads.charges("normal", n, 32)
    f = kifmm.FMM(x, 3, 5, cube=None)
    dev = torch.device("cuda:0")
    grad = torch.zeros(n, 3, device=dev)
    f.evaluate(torch.from_numpy(s).to(dev), None, grad)
    torch.cuda.synchronize()
    info = kifmm.kifmm_tree_stats_get(f.tree)
    f.close()
    c, r = info["center"], info["half_width"]
    _, rg, t, _ = oracle_evaluate(x, s, 3, 5, (c[0], c[1], c[2], r))
    assert_parity("grad", grad.cpu().double().numpy(), rg, leaf_groups(t), TOL)


def test_coincident_and_grid_aligned_points():
    # Duplicated points (pairs at zero distance contribute nothing, on both sides) and
    # points on leaf faces and on the cube's top faces (assigned to the last box).
    log("coincident and grid-aligned points")
    rng = np.random.default_rng(31)
    base = workloads.points("cube", 6_000, 30)
    dup = base[rng.choice(len(base), 500, replace=False)]
    grid = (rng.integers(0, 9, size=(300, 3)) / 8.0).astype(np.float32)   # k/8 in [0, 1], 1.0 included
    x = np.concatenate([base, dup, grid]).astype(np.float32)
    s = workloads.charges("uniform11", len(x), 32)
    phi, g, f = gpu_evaluate(x, s, 3, 5, UNIT)
    f.close()
    assert np.isfinite(phi).all() and np.isfinite(g).all()
    rphi, rg, t, _ = oracle_evaluate(x, s, 3, 5, UNIT)
    assert_parity("phi", phi, rphi, leaf_groups(t), TOL)
    assert_parity("grad", g, rg, leaf_groups(t), TOL)


@pytest.mark.parametrize("depth,n,p,dist", [
    (1, 6_000, 6, "cube"),      # the direct sum: every leaf block exceeds the LDS capacity (fused kernel)
    (2, 20_000, 5, "cube"),     # far field at level 2; the U-list kernel on its own stream
    (3, 40_000, 4, "sphere"),   # dense sphere leaves: some blocks fit in LDS, others do not
])
def test_leaf_blocks_beyond_lds_capacity(depth, n, p, dist):
    # A parent's 4 x 4 x 4 leaf block holding more sources than the leaf kernel's LDS
    # capacity (about 4,100 padded sources at p = 5..6) is read from global memory instead.
    log(f"LDS overflow depth={depth} n={n} p={p} {dist}")
    x = workloads.points(dist, n, 4100 + n)
    s = workloads.charges("uniform11", n, 4200 + n)
    cube = UNIT if dist == "cube" else (0.0, 0.0, 0.0, 1.0)
    blocks = kifmm.KIFMM_LEAF_BLOCKS
    phi, g, f = gpu_evaluate(x, s, depth, p, cube, flags=blocks)
    f.close()
    if depth <= 1:
        x64, s64 = x.astype(np.float64), s.astype(np.float64)
        rphi, rg = direct.potential(x64, x64, s64), direct.gradient(x64, x64, s64)
        groups = [np.arange(n)]
    else:
        rphi, rg, t, _ = oracle_evaluate(x, s, depth, p, cube)
        groups = leaf_groups(t)
    assert_parity("phi", phi, rphi, groups, TOL)
    assert_parity("grad", g, rg, groups, TOL)


@pytest.mark.parametrize("name,n,depth,p,dist,serial", [
    ("sphere", 60_000, 5, 6, "sphere", False),     # uneven leaves: the case the work queue is for
    ("sphere_serial", 60_000, 5, 6, "sphere", True),
    ("cube", 30_000, 4, 5, "cube", False),
    ("shallow", 2_000, 1, 4, "cube", True),        # the direct sum
])
def test_leaf_work_queue_matches_per_parent_kernel(name, n, depth, p, dist, serial):
    # The persistent work-queue kernel takes each leaf's sources in the per-parent kernel's
    # order with the same FP32 partials and FP64 accumulation: the two agree to FP32
    # rounding, and both match the oracle.  The per-parent kernel's result does not depend
    # on its workgroup size (256 or 320 threads): the same bits.
    log(f"leaf queue {name} n={n} depth={depth} p={p} serial={serial}")
    x = workloads.points(dist, n, 4300 + n)
    s = workloads.charges("normal", n, 4400 + n)
    cube = UNIT if dist == "cube" else (0.0, 0.0, 0.0, 1.0)
    out = {}
    fixed = kifmm.KIFMM_NO_AUTOTUNE   # the same M2L slab for the bitwise comparison
    for label, fl in (("queue", kifmm.KIFMM_LEAF_QUEUE),
                      ("blocks320", kifmm.KIFMM_LEAF_BLOCKS | kifmm.KIFMM_LEAF_THREADS_320 | fixed),
                      ("blocks256", kifmm.KIFMM_LEAF_BLOCKS | kifmm.KIFMM_LEAF_THREADS_256 | fixed)):
        phi, g, f = gpu_evaluate(x, s, depth, p, cube, serial=serial, flags=fl)
        st = kifmm.kifmm_plan_get_stats(f.plan)
        f.close()
        assert st["leaf_queue"] == (1 if label == "queue" else 0)
        if label != "queue":
            assert st["p2p_threads"] == int(label[-3:])
        else:
            assert st["leaf_tiles"] >= 1
        out[label] = (phi, g)
    np.testing.assert_array_equal(out["blocks256"][0], out["blocks320"][0])
    np.testing.assert_array_equal(out["blocks256"][1], out["blocks320"][1])
    assert rel_l2(out["queue"][0], out["blocks320"][0]) < 1e-6
    assert rel_l2(out["queue"][1], out["blocks320"][1]) < 1e-6
    rphi, rg, t, _ = oracle_evaluate(x, s, depth, p, cube)
    assert_parity("phi (queue)", out["queue"][0], rphi, leaf_groups(t), TOL)
    assert_parity("grad (queue)", out["queue"][1], rg, leaf_groups(t), TOL)


@pytest.mark.parametrize("per_parent,serial", [(5, False), (5, True), (15, False), (15, True),
                                               (28, False), (28, True)])
def test_short_waves_split_over_lanes(per_parent, serial):
    # A wave of the per-parent leaf kernel holding nt <= 32 targets gives each target 2, 3 or
    # 9 lanes (nt <= 32, 21, 7), each summing a share of the target's nine source runs, the
    # shares added in a fixed order.  Depth 3 (64 parents) with about `per_parent` points per
    # parent: nearly every parent is one such wave.  Against the oracle, and the same bits at
    # 256 and 320 threads (near field alone and then the far field, or fused when serial).
    n = 64 * per_parent
    log(f"short waves n={n} serial={serial}")
    x = workloads.points("cube", n, 4600 + n)
    s = workloads.charges("normal", n, 4700 + n)
    out = {}
    for threads, fl in ((320, kifmm.KIFMM_LEAF_THREADS_320), (256, kifmm.KIFMM_LEAF_THREADS_256)):
        phi, g, f = gpu_evaluate(x, s, 3, 5, UNIT, serial=serial,
                                 flags=fl | kifmm.KIFMM_LEAF_BLOCKS | kifmm.KIFMM_NO_AUTOTUNE)
        st = kifmm.kifmm_plan_get_stats(f.plan)
        f.close()
        assert st["p2p_threads"] == threads and st["leaf_queue"] == 0
        out[threads] = (phi, g)
    np.testing.assert_array_equal(out[256][0], out[320][0])
    np.testing.assert_array_equal(out[256][1], out[320][1])
    rphi, rg, t, _ = oracle_evaluate(x, s, 3, 5, UNIT)
    per_parent_targets = {}
    for leaf, idx in t.leaf_points.items():
        key = tuple(int(v) // 2 for v in leaf)
        per_parent_targets[key] = per_parent_targets.get(key, 0) + len(idx)
    assert any(0 < c % 64 <= 32 for c in per_parent_targets.values())   # split waves occur
    assert_parity("phi", out[320][0], rphi, leaf_groups(t), TOL)
    assert_parity("grad", out[320][1], rg, leaf_groups(t), TOL)


def test_device_tree_build_and_plan_on_a_stream():
    # The tree built from device points (copied on a stream), the plan created on that
    # stream and evaluated on it, with non-default surface radii; against the oracle with
    # the same radii.
    import torch
    log("device tree build, plan on a stream, alpha 1.2 / 2.7")
    n = 12_000
    x = workloads.points("cube", n, 4501)
    s = workloads.charges("uniform01", n, 4502)
    dev = torch.device("cuda:0")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        xd = torch.from_numpy(x).to(dev)
        f = kifmm.FMM(xd, 3, 5, cube=UNIT, stream=st.cuda_stream, alpha_inner=1.2, alpha_outer=2.7)
        sd = torch.from_numpy(s).to(dev)
        pot = torch.full((n,), float("nan"), device=dev)
        grad = torch.full((n, 3), float("nan"), device=dev)
        f.evaluate(sd, pot, grad, stream=st.cuda_stream)
    st.synchronize()
    order = kifmm.kifmm_tree_get_order(f.tree, n)
    f.close()
    from oracle import fmm, operators, tree
    t = tree.Tree(x.astype(np.float64), 3, UNIT[:3], UNIT[3])
    np.testing.assert_array_equal(order, t.order)
    ops = operators.Operators(5, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6, alpha_inner=1.2, alpha_outer=2.7)
    rphi, rg = fmm.evaluate(t, ops, s.astype(np.float64))
    assert_parity("phi", pot.cpu().double().numpy(), rphi, leaf_groups(t), TOL)
    assert_parity("grad", grad.cpu().double().numpy(), rg, leaf_groups(t), TOL)


def test_destroyed_plan_and_capability_errors():
    import torch
    log("handle states and plan capabilities")
    x = workloads.points("cube", 3000, 4601)
    dev = torch.device("cuda:0")
    sd = torch.ones(3000, device=dev)
    pot = torch.zeros(3000, device=dev)
    grad = torch.zeros(3000, 3, device=dev)
    f = kifmm.FMM(x, 3, 4, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL)
    with pytest.raises(kifmm.KifmmError) as e:
        f.evaluate(sd, pot, grad)   # no KIFMM_GRADIENT
    assert e.value.status == kifmm.KIFMM_E_STATE
    with pytest.raises(kifmm.KifmmError) as e:
        f.vjp(sd, sd, None, pot, None)   # no KIFMM_VJP
    assert e.value.status == kifmm.KIFMM_E_STATE
    # the plan keeps its tree and operators: destroying their handles first is allowed
    kifmm.kifmm_tree_destroy(f.tree)
    kifmm.kifmm_ops_destroy(f.ops)
    f.tree = f.ops = None
    f.evaluate(sd, pot)
    torch.cuda.synchronize()
    assert np.isfinite(pot.cpu().numpy()).all()
    plan = f.plan
    kifmm.kifmm_plan_destroy(plan)
    f.plan = None
    with pytest.raises(kifmm.KifmmError) as e:
        kifmm.kifmm_evaluate(plan, sd, pot)
    assert e.value.status == kifmm.KIFMM_E_STATE
    with pytest.raises(kifmm.KifmmError) as e:
        kifmm.kifmm_plan_destroy(plan)
    assert e.value.status == kifmm.KIFMM_E_STATE
