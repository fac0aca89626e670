"""The full-size precision, batching and differentiation workloads against the FP64
oracle on sampled leaves.

The oracle's values (Algorithm 1 with the Table 1 operators, FP64: the full upward
pass, then the downward and leaf passes of the sampled leaves and their ancestors) are
stored in tests/golden/fullsize_<workload>.npz by tests/golden/make_fullsize_oracle.py,
which calls only oracle/ on the seeded inputs of the workload generator: the oracle needs
minutes per workload, too long to run inside a GPU test.  Each file also holds the direct
sum of eq. (1) at the same points, so the approximation error of the kiFMM itself is on
record beside the GPU's parity with the oracle.

Tolerances (relative L2 against the oracle, over all sampled points and, times 10, over
each sampled leaf): 1e-6 for the plain FP32 path; 1e-5, the reduced-precision bar, for the
split-bfloat16 M2L forms, with the six-product form's accuracy against the direct sum
also required to equal FP32's (within 25 %).  The
self-comparisons at the end of each test (forms against each other, columns against
single-RHS evaluates, the derivative against its definition) are further checks, not the
parity evidence.
"""

import os

import numpy as np
import pytest

from gpu_helpers import assert_parity, log, rel_l2
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    g = np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"), allow_pickle=False)
    w = workloads.WORKLOADS[name]
    assert str(g["workload"]) == name and int(g["n"]) == w.n and int(g["p"]) == w.p and int(g["depth"]) == w.depth
    leaf_of = g["leaf_of"]
    groups = [np.flatnonzero(leaf_of == i) for i in range(len(g["leaves"]))]
    return g, w, groups


def _setup(w, nrhs, flags):
    x, s = workloads.make(w)
    c = w.cube[0] + (w.cube[1],)
    tree = kifmm.kifmm_tree_build_host(x, w.depth, c)
    ops = kifmm.kifmm_ops_precompute(w.p, eps_pinv=1e-7, eps_svd=-float(w.m2l_rank) if w.m2l_rank else 1e-6)
    return x, s, tree, ops


def _run(tree, ops, nrhs, flags, charges, want_grad):
    import torch
    plan = kifmm.kifmm_plan_create(tree, ops, nrhs, flags)
    dev = torch.device("cuda:0")
    n = charges.shape[0]
    sd = torch.from_numpy(charges).to(dev)
    pot = torch.full(charges.shape, float("nan"), device=dev)
    grad = torch.full((n, 3), float("nan"), device=dev) if want_grad else None
    kifmm.kifmm_evaluate(plan, sd, pot, grad, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    stats = kifmm.kifmm_plan_get_stats(plan)
    kifmm.kifmm_plan_destroy(plan)
    return pot.cpu().double().numpy(), (None if grad is None else grad.cpu().double().numpy()), stats


def test_precision_workload_fp32_and_split_bf16():
    # 8,000,000 points, p = 8, depth 6, N(0,1) charges, potentials: FP32, bf16x3, bf16x6.
    g, w, groups = _golden("cube8m_p8_d6")
    log(f"precision workload {w.name}: {len(groups)} sampled leaves, {len(g['idx'])} points")
    x, s, tree, ops = _setup(w, 1, 0)
    assert kifmm.kifmm_ops_get_info(ops)["rank_m2l"] == int(g["rank_m2l"])
    idx, ref, direct_ref = g["idx"], g["phi"], g["direct_phi"]
    phi = {}
    try:
        # both split-bfloat16 forms are held to the reduced-precision bar here; on the smaller
        # cases of test_gpu_split_bf16.py the six-product form meets the FP32 bar as well
        for m2l, fl, tol in (("fp32", 0, 1e-6), ("bf16x3", kifmm.KIFMM_M2L_BF16X3, 1e-5),
                             ("bf16x6", kifmm.KIFMM_M2L_BF16X6, 1e-5)):
            log(f"  {m2l}")
            phi[m2l], _, _ = _run(tree, ops, 1, kifmm.KIFMM_POTENTIAL | fl, s, False)
            assert np.isfinite(phi[m2l]).all()
            assert_parity(f"{m2l} phi vs oracle", phi[m2l][idx], ref, groups, tol)
    finally:
        kifmm.kifmm_ops_destroy(ops)
        kifmm.kifmm_tree_destroy(tree)
    e_dir = {m: rel_l2(v[idx], direct_ref) for m, v in phi.items()}
    log("  vs the direct sum: oracle {:.3e}, ".format(rel_l2(ref, direct_ref))
        + ", ".join(f"{m} {v:.3e}" for m, v in e_dir.items()))
    assert e_dir["bf16x6"] < 1.25 * e_dir["fp32"]   # equal accuracy: the speedup is compared at it
    for m in ("bf16x3", "bf16x6"):                   # every point, against the FP32 path
        assert rel_l2(phi[m], phi["fp32"]) < 1e-5


def test_batching_workload_32_right_hand_sides():
    # 4,000,000 points on the unit sphere, depth 7, 32 N(0,1) right-hand sides, potentials.
    g, w, groups = _golden("sphere4m_p6_d7_r32")
    log(f"batching workload {w.name}: {len(groups)} sampled leaves, {len(g['idx'])} points x 32")
    x, s, tree, ops = _setup(w, 32, 0)
    try:
        phi, _, st = _run(tree, ops, 32, kifmm.KIFMM_POTENTIAL, s, False)
        assert st["nrhs"] == 32 and np.isfinite(phi).all()
        idx, ref = g["idx"], g["phi"]
        assert ref.shape == (len(idx), 32)
        assert_parity("32 right-hand sides vs oracle", phi[idx], ref, groups, 1e-6)
        worst_col = max(rel_l2(phi[idx, r], ref[:, r]) for r in range(32))
        log(f"  worst column {worst_col:.3e}; vs the direct sum {rel_l2(phi[idx], g['direct_phi']):.3e} "
            f"(oracle {rel_l2(ref, g['direct_phi']):.3e})")
        assert worst_col < 1e-6
        # a column against a one-RHS evaluate of the same charges (the per-parent and the
        # work-queue leaf kernels, as plan creation chooses)
        p1, _, _ = _run(tree, ops, 1, kifmm.KIFMM_POTENTIAL, np.ascontiguousarray(s[:, 5]), False)
        assert rel_l2(phi[:, 5], p1) < 1e-6
    finally:
        kifmm.kifmm_ops_destroy(ops)
        kifmm.kifmm_tree_destroy(tree)


def test_differentiation_workload_forward_and_backward():
    # 2,000,000 points, p = 7, depth 6, charges U[-1,1), weights N(0,1): the forward
    # potentials and field, and the derivative of L = sum w_i f_i (charges and points).
    import torch
    g, w, groups = _golden("cube2m_p7_d6")
    log(f"differentiation workload {w.name}: {len(groups)} sampled leaves, {len(g['idx'])} points")
    x, s, tree, ops = _setup(w, 1, 0)
    wts = workloads.charges("normal", w.n, w.seed + 2000)
    flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT | kifmm.KIFMM_VJP
    plan = kifmm.kifmm_plan_create(tree, ops, 1, flags)
    try:
        dev = torch.device("cuda:0")
        sd, wd = torch.from_numpy(s).to(dev), torch.from_numpy(wts).to(dev)
        pot = torch.empty(w.n, device=dev)
        fs = torch.empty(w.n, 3, device=dev)
        gc = torch.empty(w.n, device=dev)
        gp = torch.empty(w.n, 3, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        kifmm.kifmm_evaluate(plan, sd, pot, fs, stream)
        kifmm.kifmm_evaluate_vjp(plan, sd, wd, None, gc, gp, stream)
        pw = torch.empty(w.n, device=dev)
        fw = torch.empty(w.n, 3, device=dev)
        kifmm.kifmm_evaluate(plan, wd, pw, fw, stream)
        torch.cuda.synchronize()
    finally:
        kifmm.kifmm_plan_destroy(plan)
        kifmm.kifmm_ops_destroy(ops)
        kifmm.kifmm_tree_destroy(tree)
    pot, fs, gc, gp = (t.cpu().double().numpy() for t in (pot, fs, gc, gp))
    idx = g["idx"]
    assert_parity("phi vs oracle", pot[idx], g["phi"], groups, 1e-6)
    assert_parity("grad phi vs oracle", fs[idx], g["grad"], groups, 1e-6)
    assert_parity("dL/ds vs oracle", gc[idx], g["grad_charges"], groups, 1e-6)
    assert_parity("dL/dx vs oracle", gp[idx], g["grad_points"], groups, 1e-6)
    # Against the direct-sum derivative, the GPU's error is the oracle's own truncation
    # error for gradients at p = 7 (recorded in the golden file) plus FP32 rounding.
    e_or = rel_l2(g["grad_points"], g["direct_grad_points"])
    e_gpu = rel_l2(gp[idx], g["direct_grad_points"])
    log(f"  dL/dx vs the direct-sum derivative: oracle {e_or:.3e}, GPU {e_gpu:.3e}")
    assert abs(e_gpu - e_or) < 1e-6
    # the product against its definition from two evaluates, on every point
    s64, w64 = s.astype(np.float64), wts.astype(np.float64)
    comb = w64[:, None] * fs + s64[:, None] * fw.cpu().double().numpy()
    assert rel_l2(gp, comb) < 1e-6
    np.testing.assert_array_equal(gc, pw.cpu().double().numpy())
