"""The split-bfloat16 M2L (KIFMM_M2L_BF16X3, KIFMM_M2L_BF16X6) against the FP64
oracle (the full-size precision workload is in test_gpu_fullsize.py).

Tolerances.  Three products of two-piece operands (bf16x3) leave a relative
error of about 3 * 2^-16 per product term, random in sign over the k-term sums
and the ~189 translations that feed each box; the reduced-precision bar,
relative L2 <= 1e-5, applies.  Six products of three-piece operands (bf16x6)
drop only terms of order 2^-24, the rounding level of FP32, and are held to the
plain FP32 bar, 1e-6.
"""

import numpy as np
import pytest

from gpu_helpers import assert_parity, gpu_evaluate, leaf_groups, log, oracle_evaluate, rel_l2
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

TOL = {"bf16x3": 1e-5, "bf16x6": 1e-6}
UNIT = (0.5, 0.5, 0.5, 0.5)
CASES = [
    ("cube20k_p6_d3", 20_000, 3, 6, "cube", "uniform01", False, 0),
    ("p8_normal", 40_000, 4, 8, "cube", "normal", False, 0),      # the precision workload's order and charges
    ("p8_normal_serial", 40_000, 4, 8, "cube", "normal", True, 0),
    ("ragged_p5", 7_777, 4, 5, "cube", "uniform11", False, 0),    # k = 56 -> 64
    ("sphere", 30_000, 4, 6, "sphere", "uniform01", False, 0),
    ("p2", 3_000, 3, 2, "cube", "uniform01", False, 0),            # k = 8 -> 16: one chunk, half of it padding
    ("rank94", 40_000, 4, 6, "cube", "uniform01", False, 94),     # k = 94 -> 96: three row blocks
    ("depth2", 5_000, 2, 5, "cube", "uniform11", False, 0),       # far field at level 2 only
]


@pytest.mark.parametrize("m2l", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("name,n,depth,p,dist,charges,serial,rank", CASES)
def test_split_bf16_parity_with_oracle(m2l, name, n, depth, p, dist, charges, serial, rank):
    log(f"{m2l} parity {name} n={n} depth={depth} p={p} rank={rank}")
    x = workloads.points(dist, n, 1001 if name.startswith("cube20k") else 300 + n + p)
    s = workloads.charges(charges, n, 2001 if name.startswith("cube20k") else 400 + n + p)
    cube = UNIT if dist == "cube" else (0.0, 0.0, 0.0, 1.0)
    phi, g, f = gpu_evaluate(x, s, depth, p, cube, serial=serial, m2l=m2l, rank=rank)
    k = kifmm.kifmm_ops_get_info(f.ops)["rank_m2l"]
    f.close()
    rphi, rg, t, _ = oracle_evaluate(x, s, depth, p, cube, rank=rank or None)
    assert_parity(f"{m2l} phi (k={k})", phi, rphi, leaf_groups(t), TOL[m2l])
    assert_parity(f"{m2l} grad", g, rg, leaf_groups(t), TOL[m2l])


@pytest.mark.parametrize("m2l", ["bf16x3", "bf16x6"])
def test_split_bf16_repeatable_and_linear(m2l):
    log(f"{m2l} determinism/linearity")
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    x, s1 = workloads.make(w)
    s2 = workloads.charges("normal", len(x), 98)
    c = w.cube[0] + (w.cube[1],)
    p1, g1, f = gpu_evaluate(x, s1, w.depth, w.p, c, m2l=m2l)
    p1b, g1b, _ = gpu_evaluate(x, s1, w.depth, w.p, c, fmm_obj=f)
    np.testing.assert_array_equal(p1, p1b)
    np.testing.assert_array_equal(g1, g1b)
    p2, g2, _ = gpu_evaluate(x, s2, w.depth, w.p, c, fmm_obj=f)
    s12 = (0.5 * s1.astype(np.float64) - 2.0 * s2.astype(np.float64)).astype(np.float32)
    p12, g12, _ = gpu_evaluate(x, s12, w.depth, w.p, c, fmm_obj=f)
    f.close()
    assert rel_l2(p12, 0.5 * p1 - 2.0 * p2) < 1e-5
    assert rel_l2(g12, 0.5 * g1 - 2.0 * g2) < 1e-5


def test_split_bf16_rejects_both_forms():
    x = workloads.points("cube", 100, 5)
    with pytest.raises(kifmm.KifmmError):
        kifmm.FMM(x, 2, 3, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_M2L_BF16X3 | kifmm.KIFMM_M2L_BF16X6)
