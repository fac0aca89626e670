"""Several right-hand sides in one evaluate (plans with nrhs > 1, potentials
only) against the FP64 oracle, which takes [N, R] charges, and against one
single-RHS evaluate per column.

Tolerance: relative L2 <= 1e-6 against the oracle (plain FP32 path), per
right-hand side.
"""

import numpy as np
import pytest

from gpu_helpers import assert_parity, gpu_evaluate, leaf_groups, log, oracle_evaluate, rel_l2
from oracle import direct
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6
UNIT = (0.5, 0.5, 0.5, 0.5)
SPHERE = (0.0, 0.0, 0.0, 1.0)


def _charges(n, R, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, R)).astype(np.float32)


@pytest.mark.parametrize("name,n,depth,p,dist,R,m2l,rank", [
    ("cube20k_p6_d3", 20_000, 3, 6, "cube", 4, "fp32", 0),
    ("cube20k_p6_d3_r32", 20_000, 3, 6, "cube", 32, "fp32", 0),
    ("sphere_r8", 30_000, 4, 6, "sphere", 8, "fp32", 0),
    ("ragged_r2", 7_777, 4, 5, "cube", 2, "fp32", 0),
    ("sparse_deep_r16", 2_000, 5, 4, "cube", 16, "fp32", 0),
    ("cube20k_r4_bf16x6", 20_000, 3, 6, "cube", 4, "bf16x6", 0),
    ("sphere_r32_rank94", 30_000, 4, 6, "sphere", 32, "fp32", 94),   # wide M2L, three row blocks
    ("ragged_r32_p5", 7_777, 4, 5, "cube", 32, "fp32", 0),     # n = 98: four check blocks, a partial float4
    ("sparse_deep_r32_p4", 2_000, 5, 4, "cube", 32, "fp32", 0),  # n = 56: two check blocks, long U2U chains
])
def test_multi_rhs_parity_with_oracle(name, n, depth, p, dist, R, m2l, rank):
    log(f"multi-RHS parity {name} n={n} depth={depth} p={p} R={R} {m2l} rank={rank}")
    x = workloads.points(dist, n, 1001 if name.startswith("cube20k") else 800 + n)
    s = _charges(n, R, 900 + n + R)
    cube = UNIT if dist == "cube" else SPHERE
    phi, _, f = gpu_evaluate(x, s, depth, p, cube, gradient=False, m2l=m2l, rank=rank)
    assert kifmm.kifmm_plan_get_stats(f.plan)["nrhs"] == R
    f.close()
    rphi, _, t, _ = oracle_evaluate(x, s, depth, p, cube, gradient=False, rank=rank or None)
    errs = [rel_l2(phi[:, r], rphi[:, r]) for r in range(R)]
    log(f"  rel-L2 per right-hand side: max {max(errs):.3e} mean {np.mean(errs):.3e}")
    assert max(errs) < TOL
    assert_parity("all right-hand sides", phi, rphi, leaf_groups(t), TOL)


def test_multi_rhs_columns_match_single_rhs():
    log("multi-RHS columns vs single-RHS evaluates")
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    x, _ = workloads.make(w)
    c = w.cube[0] + (w.cube[1],)
    R = 8
    s = _charges(len(x), R, 77)
    phi, _, f = gpu_evaluate(x, s, w.depth, w.p, c, gradient=False)
    f.close()
    single = None
    for r in (0, 3, 7):
        p1, _, single = gpu_evaluate(x, s[:, r], w.depth, w.p, c, gradient=False, fmm_obj=single)
        e = rel_l2(phi[:, r], p1)
        log(f"  column {r}: rel-L2 vs single {e:.3e}")
        assert e < 3e-7
    single.close()


def test_multi_rhs_shallow_tree_is_direct_sum():
    log("multi-RHS depth 1 = direct sum")
    n, R = 1500, 4
    x = workloads.points("cube", n, 55)
    s = _charges(n, R, 56)
    phi, _, f = gpu_evaluate(x, s, 1, 4, UNIT, gradient=False)
    f.close()
    x64 = x.astype(np.float64)
    ref = direct.potential(x64, x64, s.astype(np.float64))
    assert rel_l2(phi, ref) < TOL


def test_multi_rhs_argument_errors():
    import torch
    x = workloads.points("cube", 400, 57)
    with pytest.raises(kifmm.KifmmError):   # gradients need nrhs = 1
        kifmm.FMM(x, 2, 3, cube=UNIT, nrhs=4)
    with pytest.raises(kifmm.KifmmError):   # unsupported count
        kifmm.FMM(x, 2, 3, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL, nrhs=3)
    f = kifmm.FMM(x, 2, 3, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL, nrhs=4)
    dev = torch.device("cuda:0")
    with pytest.raises(kifmm.KifmmError):   # potentials must be requested
        f.evaluate(torch.zeros(400, 4, device=dev), None, torch.zeros(400, 3, device=dev))
    f.close()
