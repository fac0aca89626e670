"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs."""

import sys

import numpy as np

from oracle import direct, fmm, operators, tree
from paper_2604_19243_amd import kifmm


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


M2L_FLAGS = {"fp32": 0, "bf16x3": kifmm.KIFMM_M2L_BF16X3, "bf16x6": kifmm.KIFMM_M2L_BF16X6,
             "blocked": kifmm.KIFMM_M2L_BLOCKED, "gather": kifmm.KIFMM_M2L_GATHER}


def gpu_evaluate(points, charges, depth, p, cube, eps_svd=1e-6, rank=0, gradient=True, fmm_obj=None, serial=False,
                 m2l="fp32", flags=0):
    """HIP path: returns (phi [n] or [n,R], grad [n,3] or None, FMM object) as float64 numpy arrays.
    charges [n] or [n, R] (R right-hand sides: potentials only); `flags`: further plan flags."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrhs = 1 if np.ndim(charges) == 1 else np.shape(charges)[1]
    flags |= (kifmm.KIFMM_POTENTIAL | (kifmm.KIFMM_GRADIENT if gradient else 0) | (kifmm.KIFMM_SERIAL if serial else 0)
              | M2L_FLAGS[m2l])
    f = fmm_obj or kifmm.FMM(points, depth, p, cube=cube, eps_svd=eps_svd, rank=rank, flags=flags, nrhs=nrhs)
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(charges, dtype=np.float32)).to(dev)
    pot = torch.full(np.shape(charges), float("nan"), device=dev)
    grad = torch.full((len(points), 3), float("nan"), device=dev) if gradient else None
    f.evaluate(s, pot, grad, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return (pot.cpu().double().numpy(), None if grad is None else grad.cpu().double().numpy(), f)


def oracle_evaluate(points, charges, depth, p, cube, eps_svd=1e-6, rank=None, gradient=True, target_leaves=None):
    t = tree.Tree(np.asarray(points, dtype=np.float64), depth, cube[:3], cube[3])
    ops = operators.Operators(p, eps_pinv=1e-7, m2l="compressed", eps_svd=eps_svd, rank=rank)
    phi, g = fmm.evaluate(t, ops, np.asarray(charges, dtype=np.float64), gradient=gradient,
                          target_leaves=target_leaves)
    return phi, g, t, ops


rel_l2 = direct.rel_l2


def leaf_groups(t, leaves=None):
    """Input indices of the points of each non-empty leaf of the oracle tree `t` (or of the given leaves)."""
    if leaves is None:
        return list(t.leaf_points.values())
    return [t.leaf_points[tuple(int(v) for v in b)] for b in leaves if tuple(int(v) for v in b) in t.leaf_points]


def assert_parity(label, gpu, ref, groups, tol):
    """Relative L2 over the points of `groups` <= tol, and per group (leaf) <= 10 tol, so that an error
    confined to a few leaves is not diluted by all the others.

    A leaf's error is taken relative to its own norm, floored at its share of the whole norm,
    |ref| sqrt(m / M) for m of the M points: where a leaf's values happen to nearly cancel (one or
    two points with signed charges), its own norm is no scale for FP32 rounding made in sums of
    many terms."""
    idx = np.concatenate(groups)
    e = rel_l2(gpu[idx], ref[idx])
    total = np.linalg.norm(np.asarray(ref[idx], dtype=np.float64).ravel())
    worst = 0.0
    for g in groups:
        if not len(g):
            continue
        err = np.linalg.norm((np.asarray(gpu[g], dtype=np.float64) - ref[g]).ravel())
        floor = total * np.sqrt(len(g) / len(idx))
        worst = max(worst, err / max(np.linalg.norm(np.asarray(ref[g], dtype=np.float64).ravel()), floor))
    log(f"  {label}: rel-L2 {e:.3e}, worst leaf {worst:.3e} ({len(groups)} leaves, {len(idx)} points)")
    assert e < tol, (label, e)
    assert worst < 10 * tol, (label, worst)
    return e, worst
