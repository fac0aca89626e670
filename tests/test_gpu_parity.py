"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded inputs.

Tolerance: relative L2 <= 1e-6 for potentials and gradients of the plain FP32 path.
"""

import numpy as np
import pytest

from gpu_helpers import gpu_evaluate, log, oracle_evaluate, rel_l2
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
    rphi, rg, _, ops = oracle_evaluate(x, s, depth, p, cube, rank=rank or None)
    assert ops.compression(1.0)[0].shape[1] == k
    e, eg = rel_l2(phi, rphi), rel_l2(g, rg)
    log(f"  rel-L2 phi {e:.3e} grad {eg:.3e} (k={k})")
    assert e < TOL and eg < TOL


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
    idx = np.concatenate([t.leaf_points[b] for b in leaves if b in t.leaf_points])
    e, eg = rel_l2(phi[idx], rphi[idx]), rel_l2(g[idx], rg[idx])
    log(f"  sampled {len(idx)} points: rel-L2 phi {e:.3e} grad {eg:.3e}")
    assert e < TOL and eg < TOL


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
    rphi, rg, _, ops = oracle_evaluate(x, s, depth, p, UNIT)
    assert ops.compression(1.0)[0].shape[1] == k
    e, eg = rel_l2(phi, rphi), rel_l2(g, rg)
    log(f"  rel-L2 phi {e:.3e} grad {eg:.3e} (k={k})")
    assert e < TOL and eg < TOL


def test_orders_above_8_need_a_shallow_tree():
    # p = 9 (386 surface points): the leaf kernels hold at most 304, so a tree with a far
    # field is refused with KIFMM_E_INVALID; at depth 1 (the direct sum) the order is unused.
    log("order p=9")
    x = workloads.points("cube", 3_000, 709)
    s = workloads.charges("uniform11", 3_000, 809)
    ops = kifmm.kifmm_ops_precompute(9)
    try:
        for depth, ok in ((3, False), (1, True)):
            tree = kifmm.kifmm_tree_build(x, depth, UNIT)
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
    rphi, rg, _, _ = oracle_evaluate(x, s, depth, 4, (0.0, 0.0, 0.0, 1.0))
    e, eg = rel_l2(phi, rphi), rel_l2(g, rg)
    log(f"  rel-L2 phi {e:.3e} grad {eg:.3e}")
    assert e < TOL and eg < TOL


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
    info = kifmm.kifmm_tree_get_info(f.tree)
    f.close()
    c, r = info["center"], info["half_width"]
    _, rg, _, _ = oracle_evaluate(x, s, 3, 5, (c[0], c[1], c[2], r))
    eg = rel_l2(grad.cpu().double().numpy(), rg)
    log(f"  rel-L2 grad {eg:.3e}")
    assert eg < TOL


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
    rphi, rg, _, _ = oracle_evaluate(x, s, 3, 5, UNIT)
    e, eg = rel_l2(phi, rphi), rel_l2(g, rg)
    log(f"  rel-L2 phi {e:.3e} grad {eg:.3e}")
    assert e < TOL and eg < TOL
