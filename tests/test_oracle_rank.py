"""The M2L compression rank of the p = 6 GPU workloads (94, against 116 from the
1e-6 singular-value threshold): a rank that keeps whole clusters of equal
singular values, and whose truncation adds a bounded share to the FMM's error
against the direct sum (its definition).  The compressed operator's error is
bounded by the first dropped singular value (Section 2.2, BLAS M2L reading);
here its effect on the evaluate is measured against the uncompressed M2L and
the direct sum.
"""

import numpy as np
import pytest

from oracle import direct, fmm, operators, tree
from paper_2604_19243_amd import workloads

P6_WORKLOADS = [w for w in workloads.WORKLOADS.values() if w.p == 6 and w.m2l_rank]


def test_p6_workload_rank_keeps_clusters():
    assert P6_WORKLOADS
    ops = operators.Operators(6, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)
    _, _, _, (sf, st) = ops.compression(0.25)
    for w in P6_WORKLOADS:
        k = w.m2l_rank
        assert k <= 96 and not operators.splits_cluster(sf, k) and not operators.splits_cluster(st, k)
        # the oracle keeps the requested rank as it is
        r = operators.Operators(6, eps_pinv=1e-7, m2l="compressed", rank=k)
        assert r.compression(0.25)[0].shape[1] == k
        # the first dropped singular value is below 4.1e-6 of the largest
        assert sf[k] / sf[0] < 4.1e-6


def test_p6_workload_rank_accuracy_against_direct_sum():
    # 60,000 points uniform in the cube, depth 4 (~15 points per leaf), U[0,1) charges; the
    # points of 16 random leaves against the direct sum.  Measured on three seeds: rank 94
    # raises the error of the uncompressed M2L by 4.5-13 % here (by 1.4 % at 1M points,
    # depth 5), the 1e-6 threshold (rank 116) by at most 0.6 %.
    k = P6_WORKLOADS[0].m2l_rank
    n, depth, seed = 60_000, 4, 31
    x = workloads.points("cube", n, seed).astype(np.float64)
    s = workloads.charges("uniform01", n, seed + 1).astype(np.float64)
    t = tree.Tree(x, depth, (0.5, 0.5, 0.5), 0.5)
    rng = np.random.default_rng(seed + 2)
    all_leaves = list(t.leaf_points)
    leaves = [all_leaves[i] for i in rng.choice(len(all_leaves), 16, replace=False)]
    idx = np.concatenate([t.leaf_points[b] for b in leaves])
    ref = direct.potential(x[idx], x, s)
    err = {}
    for name, ops in (("plain", operators.Operators(6, eps_pinv=1e-7, m2l="plain")),
                      ("eps", operators.Operators(6, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6)),
                      ("rank", operators.Operators(6, eps_pinv=1e-7, m2l="compressed", rank=k))):
        phi, _ = fmm.evaluate(t, ops, s, gradient=False, target_leaves=leaves)
        err[name] = direct.rel_l2(phi[idx], ref)
    assert err["plain"] < 4e-7
    assert err["eps"] < 1.02 * err["plain"]
    assert err["rank"] < 1.2 * err["plain"]
