"""The split-bfloat16 M2L (KIFMM_M2L_BF16X3, KIFMM_M2L_BF16X6) against the FP64
oracle and against the plain FP32 path.

Tolerances.  Three products of two-piece operands (bf16x3) leave a relative
error of about 3 * 2^-16 per product term, random in sign over the k-term sums
and the ~189 translations that feed each box; the reduced-precision bar,
relative L2 <= 1e-5, applies.  Six products of three-piece operands (bf16x6)
drop only terms of order 2^-24, the rounding level of FP32, and are held to the
plain FP32 bar, 1e-6.
"""

import numpy as np
import pytest

from gpu_helpers import gpu_evaluate, log, oracle_evaluate, rel_l2
from oracle import direct
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
    rphi, rg, _, _ = oracle_evaluate(x, s, depth, p, cube, rank=rank or None)
    e, eg = rel_l2(phi, rphi), rel_l2(g, rg)
    log(f"  rel-L2 {m2l} phi {e:.3e} grad {eg:.3e} (k={k})")
    assert e < TOL[m2l] and eg < TOL[m2l]


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


def test_split_bf16_full_size_precision_workload():
    # 8,000,000 points, p = 8, depth 6, N(0,1) charges, potentials only: the
    # workload the split-bfloat16 M2L is measured on.  Too large for the oracle's
    # full upward pass in a test, so checked by properties that hold at any size:
    # each form against the plain FP32 path on every point, to the reduced-
    # precision bar (the FP32 path stands in for the oracle: its own error, about
    # 1e-6 here, is FP32 rounding in the same sums); and all three against the
    # direct sum (the definition) on sampled targets, where the error is the FMM's
    # truncation error plus the arithmetic's and bf16x6 must be as accurate as
    # FP32.
    w = workloads.WORKLOADS["cube8m_p8_d6"]
    log("split bf16 full size cube8m_p8_d6")
    x, s = workloads.make(w)
    c = w.cube[0] + (w.cube[1],)
    phi = {}
    for m2l in ("fp32", "bf16x3", "bf16x6"):
        phi[m2l], _, f = gpu_evaluate(x, s, w.depth, w.p, c, gradient=False, m2l=m2l)
        f.close()
        assert np.isfinite(phi[m2l]).all()
    idx = workloads.sample_indices(len(x), 128, 4003)
    x64, s64 = x.astype(np.float64), s.astype(np.float64)
    ref = np.zeros(len(idx))
    for a in range(0, len(x), 250_000):  # source blocks: 128 x 250k kernel entries at a time
        ref += direct.potential(x64[idx], x64[a:a + 250_000], s64[a:a + 250_000])
    e = {m: rel_l2(v[idx], ref) for m, v in phi.items()}
    d = {m: rel_l2(phi[m], phi["fp32"]) for m in ("bf16x3", "bf16x6")}
    log("  vs fp32: " + ", ".join(f"{m} {v:.3e}" for m, v in d.items())
        + "; vs direct sum (128 targets): " + ", ".join(f"{m} {v:.3e}" for m, v in e.items()))
    for m in ("bf16x3", "bf16x6"):
        assert d[m] < 1e-5
    assert e["bf16x6"] < 1.25 * e["fp32"]
