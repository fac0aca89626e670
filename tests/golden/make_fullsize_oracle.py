"""Writes the FP64 oracle's results on sampled leaves of the three full-size workloads.

The GPU parity tests of the precision (8M points, p = 8), batching (4M sphere points,
32 right-hand sides) and differentiation (2M points, p = 7) workloads compare the HIP
path with these values.  They come from ``oracle/`` alone (Algorithm 1 of Section 2.1 with
the operators of Table 1, FP64, single-threaded steps), run on the seeded inputs of
``paper_2604_19243_amd.workloads``: the full upward pass over every leaf, then the
downward and leaf passes for the sampled leaves and their ancestors only
(``fmm.evaluate(..., target_leaves=...)``).  The oracle needs minutes per workload, so the
values are stored rather than recomputed inside a GPU test.

Beside the oracle's values each file holds the direct sum of eq. (1) (and its derivative,
for the differentiation workload) at the same points, so that the oracle's own
approximation error at these depths is on record.

Usage:  python tests/golden/make_fullsize_oracle.py [workload ...]
Writes tests/golden/fullsize_<workload>.npz (no pickled objects; load with numpy.load).
"""

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import direct, fmm, operators, tree  # noqa: E402
from paper_2604_19243_amd import workloads  # noqa: E402

# sampled leaves per workload (seeded) and the workload's configuration number (seed 4000 + c)
SAMPLES = {"cube8m_p8_d6": (3, 20), "sphere4m_p6_d7_r32": (4, 14), "cube2m_p7_d6": (5, 24)}
EPS_PINV = 1e-7
EPS_SVD = 1e-6


def pick_leaves(t, config, count):
    """`count` random non-empty leaves plus extreme ones: the eight cube corners when
    non-empty, and the leaves holding the first point of each extreme coordinate and the
    most populated leaf."""
    rng = np.random.default_rng(4000 + config)
    keys = sorted(t.leaf_points, key=lambda b: tree.morton_key(b[0], b[1], b[2], t.depth))
    chosen = {keys[i] for i in rng.choice(len(keys), size=min(count, len(keys)), replace=False)}
    m = 2 ** t.depth - 1
    for c in range(8):
        b = (m * (c & 1), m * ((c >> 1) & 1), m * ((c >> 2) & 1))
        if b in t.leaf_points:
            chosen.add(b)
    for d in range(3):
        for fn in (np.argmin, np.argmax):
            chosen.add(tuple(int(v) for v in t.leaf_index[fn(t.points[:, d])]))
    chosen.add(max(t.leaf_points, key=lambda b: len(t.leaf_points[b])))
    return sorted(chosen, key=lambda b: tree.morton_key(b[0], b[1], b[2], t.depth))


def direct_potential(x, idx, s):
    out = 0.0
    for a in range(0, len(x), 500_000):
        out = out + direct.potential(x[idx], x[a:a + 500_000], s[a:a + 500_000])
    return out


def direct_gradient(x, idx, s):
    out = 0.0
    for a in range(0, len(x), 500_000):
        out = out + direct.gradient(x[idx], x[a:a + 500_000], s[a:a + 500_000], block=16)
    return out


def make(name):
    w = workloads.WORKLOADS[name]
    config, count = SAMPLES[name]
    t0 = time.perf_counter()
    x32, s32 = workloads.make(w)
    x, s = x32.astype(np.float64), s32.astype(np.float64)
    c, r = w.cube
    t = tree.Tree(x, w.depth, c, r)
    ops = operators.Operators(w.p, eps_pinv=EPS_PINV, m2l="compressed", eps_svd=EPS_SVD, rank=w.m2l_rank or None)
    leaves = pick_leaves(t, config, count)
    idx = np.concatenate([t.leaf_points[b] for b in leaves])
    leaf_of = np.concatenate([np.full(len(t.leaf_points[b]), i) for i, b in enumerate(leaves)])
    out = {"workload": np.array(name), "n": np.array(w.n), "p": np.array(w.p), "depth": np.array(w.depth),
           "nrhs": np.array(w.nrhs), "eps_pinv": np.array(EPS_PINV), "eps_svd": np.array(EPS_SVD),
           "leaves": np.array(leaves, dtype=np.int64), "idx": idx.astype(np.int64),
           "leaf_of": leaf_of.astype(np.int64)}
    if name == "cube2m_p7_d6":
        wts = workloads.charges("normal", w.n, w.seed + 2000).astype(np.float64)
        phi, g = fmm.evaluate(t, ops, np.stack([s, wts], axis=1), gradient=True, target_leaves=leaves)
        gc = phi[:, 1]
        gp = wts[:, None] * g[:, 0, :] + s[:, None] * g[:, 1, :]
        out.update(phi=phi[idx, 0], grad=g[idx, 0, :], grad_charges=gc[idx], grad_points=gp[idx])
        dphi = direct_potential(x, idx, np.stack([s, wts], axis=1))
        dgrad = direct_gradient(x, idx, np.stack([s, wts], axis=1))
        out.update(direct_phi=dphi[:, 0], direct_grad=dgrad[:, 0, :], direct_grad_charges=dphi[:, 1],
                   direct_grad_points=wts[idx, None] * dgrad[:, 0, :] + s[idx, None] * dgrad[:, 1, :])
    else:
        phi, g = fmm.evaluate(t, ops, s, gradient=w.gradient, target_leaves=leaves)
        out.update(phi=phi[idx])
        out.update(direct_phi=direct_potential(x, idx, s))
    out["rank_m2l"] = np.array(ops.compression(1.0)[0].shape[1])
    with open(os.path.join(ROOT, "oracle", "fmm.py"), "rb") as f:
        out["oracle_fmm_sha256_16"] = np.array(hashlib.sha256(f.read()).hexdigest()[:16])
    path = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(path, **out)
    e = direct.rel_l2(out["phi"], out["direct_phi"])
    print(f"{name}: {len(leaves)} leaves, {len(idx)} points, k={int(out['rank_m2l'])}, oracle vs direct phi {e:.3e}, "
          f"{time.perf_counter() - t0:.0f} s -> {path}", flush=True)
    if "grad_points" in out:
        print(f"  grad {direct.rel_l2(out['grad'], out['direct_grad']):.3e} grad_charges "
              f"{direct.rel_l2(out['grad_charges'], out['direct_grad_charges']):.3e} grad_points "
              f"{direct.rel_l2(out['grad_points'], out['direct_grad_points']):.3e}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(SAMPLES):
        make(name)
