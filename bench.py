#!/usr/bin/env python3
"""Throughput of one kiFMM evaluate (3D Laplace) on one MI355X.

A step is one full evaluate through the C ABI: permute, S2U (P2M), U2U, M2L
compression and VLI, post + D2D, D2T + ULI (L2P + P2P) writing potentials and
gradients in input order.  Inputs are resident in HBM before timing; tree build
and operator precompute are setup and are not timed.

Prints one JSON line: metric/value (Mpoints/s = N / time per evaluate, exactly
--steps evaluates between two events with stage timing off), the mean and spread
over --repeats such blocks, the roofline of the dominant kernel (M2L on the
matrix cores, timed with HIP events on its stream in a separate pass), the P2P
kernels' FLOP rates, the accuracy gate (GPU against the FP64 oracle on the points
of sampled leaves, and against the direct sum on sampled targets), the FP64
oracle timed on a bounded sample on the host CPU (one core and all cores), and
compact measurements of the precision, batching and differentiation workloads.

The headline value is printed as null, and the exit status is 1, when the
accuracy gate fails or could not be evaluated.
"""

import argparse
import hashlib
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 (vector and matrix), dense
PEAK_BF16_TFLOPS = 2500.0  # MI355X BF16 matrix, dense (no sparsity)
P2P_FLOPS_PER_PAIR = 20    # potential + gradient: 3 sub, 5 for r^2, 1 rsqrt, 2 potential, 1 + 8 gradient
METRIC = "Mpoints/s per kiFMM evaluate at rel-L2<=1e-5; P2P/M2L % roofline"
ORACLE_TOL = {"fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 1e-5}   # GPU against the FP64 oracle
DIRECT_TOL = 1e-5                                              # the metric's rel-L2 bar, against eq. (1)


def kernel_source_hash():
    """Hash of the M2L kernels' source (the kernels whose HBM traffic profiles/traffic.json records)."""
    with open(os.path.join(ROOT, "paper_2604_19243_amd", "csrc", "m2l.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload, kernel, config):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None if stale, missing
    or measured on another launch configuration."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            entries = json.load(f)[kernel][workload]
    except (OSError, KeyError, ValueError):
        return None
    for entry in entries if isinstance(entries, list) else [entries]:
        if entry.get("m2l_hip_sha256_16") == kernel_source_hash() and entry.get("config") == config:
            return float(entry["hbm_bytes_per_launch"])
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# --------------------------------------------------------------------------- CPU children

def leaf_parity(gpu, ref, groups):
    """Relative L2 over all sampled points and the worst leaf (its own norm floored at its
    share of the total), as in the parity tests."""
    import numpy as np
    idx = np.concatenate(groups)
    total = np.linalg.norm(ref[idx].ravel())
    e = float(np.linalg.norm((gpu[idx] - ref[idx]).ravel()) / total)
    worst = 0.0
    for g in groups:
        err = np.linalg.norm((gpu[g] - ref[g]).ravel())
        worst = max(worst, err / max(np.linalg.norm(ref[g].ravel()), total * np.sqrt(len(g) / len(idx))))
    return e, float(worst)


_SHARED = {}


def _direct_block(job):
    from oracle import direct
    kind, a, b = job
    x, s, idx = _SHARED["x"], _SHARED["s"], _SHARED["idx"]
    if kind == "potential":
        return direct.potential(x[idx], x[a:b], s[a:b], block=256)
    return direct.gradient(x[idx], x[a:b], s[a:b], block=16)


def direct_sum(kind, x, s, idx, block=100_000):
    """oracle.direct's potential or gradient at the targets x[idx] from all sources, the source
    blocks spread over the host's cores (forked workers) and added in block order."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    _SHARED.update(x=x, s=s, idx=idx)
    jobs = [(kind, a, min(a + block, len(x))) for a in range(0, len(x), block)]
    workers = max(1, min(len(jobs), len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_direct_block, jobs))
    out = parts[0]
    for part in parts[1:]:
        out = out + part
    return out


def oracle_worker(args):
    """Child process: the FP64 oracle on a bounded sample of the workload (timed), its parity with
    the GPU on the sampled leaves, and the direct sum at sampled targets."""
    import numpy as np

    from oracle import direct, fmm, operators, tree
    from paper_2604_19243_amd import workloads

    w = workloads.WORKLOADS[args.workload]
    x32, s32 = workloads.make(w)
    x, s = x32.astype(np.float64), s32.astype(np.float64)
    gpu = np.load(args.gpu_sample, allow_pickle=False)
    out = {}
    c, r = w.cube
    t = tree.Tree(x, w.depth, c, r)
    rank = w.m2l_rank if args.m2l_rank is None else args.m2l_rank
    ops = operators.Operators(w.p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6, rank=rank or None)
    L = w.depth
    for l in range(2, L + 1):
        ops.compression(t.radius(l))          # operator setup, not timed (as on the GPU)
    s2 = s[:, None] if s.ndim == 1 else s
    rng = np.random.default_rng(4000 + args.sample_seed)
    all_leaves = list(t.leaf_points)
    pick = rng.choice(len(all_leaves), size=min(args.sample_leaves, len(all_leaves)), replace=False)
    leaves = [all_leaves[i] for i in pick]
    needed = [set() for _ in range(L + 1)]
    for b in leaves:
        for l in range(L + 1):
            needed[l].add((b[0] >> (L - l), b[1] >> (L - l), b[2] >> (L - l)))
    needed = [sorted(v) for v in needed]

    t0 = time.perf_counter()
    u = fmm.upward_pass(t, ops, s2)
    t1 = time.perf_counter()
    d = fmm.downward_pass(t, ops, u, needed)
    t2 = time.perf_counter()
    phi, grad = fmm.leaf_pass(t, ops, s2, d, leaves, w.gradient)
    t3 = time.perf_counter()
    boxes_all = sum(len(t.boxes[l]) for l in range(2, L + 1))
    boxes_sampled = sum(len(needed[l]) for l in range(2, L + 1))
    t_full = (t1 - t0) + (t2 - t1) * boxes_all / boxes_sampled + (t3 - t2) * len(all_leaves) / len(leaves)
    threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    out["timing"] = {
        "value": w.n / t_full / 1e6, "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle, {threads} BLAS thread(s): full upward pass ({t1 - t0:.2f} s) timed; "
                   f"downward pass timed on the {boxes_sampled} ancestors of {len(leaves)} random leaves "
                   f"({t2 - t1:.2f} s) and leaf pass on those leaves ({t3 - t2:.2f} s), each scaled by box/leaf "
                   f"counts to the full workload; extrapolated evaluate {t_full:.1f} s"),
        "seconds_measured": t3 - t0, "seconds_extrapolated": t_full, "cpu_model": cpu_model()}
    if args.timing_only:
        print(json.dumps(out), flush=True)
        return

    # GPU against the oracle on the points of the sampled leaves
    groups = [t.leaf_points[b] for b in leaves]
    gphi = gpu["phi"].astype(np.float64)
    e, worst = leaf_parity(gphi, phi[:, 0] if gphi.ndim == 1 else phi, groups)
    out["oracle_parity"] = {"leaves": len(leaves), "points": int(sum(len(g) for g in groups)),
                            "rel_l2_phi": e, "worst_leaf_phi": worst}
    if w.gradient and "grad" in gpu:
        e, worst = leaf_parity(gpu["grad"].astype(np.float64), grad[:, 0, :], groups)
        out["oracle_parity"].update(rel_l2_grad=e, worst_leaf_grad=worst)

    # the direct sum of eq. (1) at sampled targets, sources in blocks
    idx = gpu["direct_idx"]
    ref = direct_sum("potential", x, s, idx)
    out["direct"] = {"targets": int(len(idx)), "rel_l2_phi": direct.rel_l2(gphi[idx], ref)}
    if w.gradient and "grad" in gpu:
        gidx = idx[:args.direct_grad_targets]
        gref = direct_sum("gradient", x, s, gidx)
        out["direct"].update(grad_targets=int(len(gidx)), rel_l2_grad=direct.rel_l2(gpu["grad"][gidx], gref))
    for key in gpu.files:
        if key.startswith("extra_phi_"):   # other runs of the same workload (another M2L rank or form)
            out["direct"][key[len("extra_"):]] = direct.rel_l2(gpu[key], ref)
    print(json.dumps(out), flush=True)


def direct_worker(args):
    """Child process: the direct sum of eq. (1) (or its derivative) at sampled targets of a
    workload, against the GPU values of several runs."""
    import numpy as np

    from oracle import direct
    from paper_2604_19243_amd import workloads

    w = workloads.WORKLOADS[args.workload]
    x32, s32 = workloads.make(w)
    x, s = x32.astype(np.float64), s32.astype(np.float64)
    gpu = np.load(args.gpu_sample, allow_pickle=False)
    idx = gpu["idx"]
    out = {"targets": int(len(idx))}
    if "weights" in gpu.files:
        # the derivative of sum w_i f_i: dL/ds (potential of w) and dL/dx
        wts = gpu["weights"].astype(np.float64)
        sw = np.stack([s, wts], axis=1)
        ph = direct_sum("potential", x, sw, idx)
        gr = direct_sum("gradient", x, sw, idx)
        gp = wts[idx, None] * gr[:, 0, :] + s[idx, None] * gr[:, 1, :]
        out["grad_charges"] = direct.rel_l2(gpu["grad_charges"], ph[:, 1])
        out["grad_points"] = direct.rel_l2(gpu["grad_points"], gp)
        out["phi"] = direct.rel_l2(gpu["phi"], ph[:, 0])
    else:
        ref = direct_sum("potential", x, s, idx)
        for key in gpu.files:
            if key.startswith("phi_"):
                out[key[4:]] = direct.rel_l2(gpu[key], ref)
    print(json.dumps(out), flush=True)


def run_child(mode, path, workload, extra, threads, timeout=900):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OPENBLAS_NUM_THREADS=str(threads),
               MKL_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), mode, "--workload", workload, "--gpu-sample", path] + extra
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    if r.returncode != 0:
        print(r.stderr[-3000:], file=sys.stderr, flush=True)
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


# --------------------------------------------------------------------------- GPU timing

class Timer:
    """Warm-up, then blocks of exactly `steps` steps between two events on the evaluate stream."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream

    def block(self, step, steps):
        torch = self.torch
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(self.stream)
        for _ in range(steps):
            step()
        end.record(self.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(end) / steps

    def stages(self, plan, step, steps):
        """Per-stage milliseconds per call from the plan's stage events (a separate pass)."""
        from paper_2604_19243_amd import kifmm
        kifmm.kifmm_plan_set_timing(plan, True)
        kifmm.kifmm_plan_get_stage_times(plan, reset=True)
        for _ in range(steps):
            step()
        self.torch.cuda.synchronize()
        st = kifmm.kifmm_plan_get_stage_times(plan, reset=True)
        kifmm.kifmm_plan_set_timing(plan, False)
        return {k: v[0] / max(v[1], 1) for k, v in st.items()}


def mean_std(v):
    import numpy as np
    a = np.asarray(v, dtype=np.float64)
    return float(a.mean()), float(a.std(ddof=1)) if len(a) > 1 else 0.0


def bf16_products(stats, passes):
    """bfloat16 matrix products (per V-list pair and k^2) executed by the KIFMM_STAGE_M2L launches:
    bf16x6 six per pair; bf16x3 three at the leaf level and six above it."""
    stage, leaf = stats["m2l_stage_pairs"], stats["m2l_pairs_leaf"]
    if passes == 3:
        return 3 * leaf + 6 * (stage - leaf)
    return passes * stage


def leaf_kernel_name(stats, serial, R):
    if R > 1:
        return "k_leaf_r32" if R == 32 else f"k_leaf_multi<{R}>"
    if stats["leaf_queue"]:
        return "k_leaf_queue<0>" if serial else "k_leaf_queue<1>"
    return "k_p2p<0>" if serial else "k_p2p<1>"


def next_rows(args, torch, dev):
    """Compact measurements of the precision, batching and differentiation workloads."""
    import numpy as np

    from paper_2604_19243_amd import kifmm, workloads
    rows = {}
    stream = torch.cuda.current_stream()
    tm = Timer(torch, stream)
    steps = args.next_steps

    # precision: 8M points, p = 8, depth 6, N(0,1) charges, potentials; FP32 and split bfloat16 M2L
    w = workloads.WORKLOADS["cube8m_p8_d6"]
    print(f"# next: {w.name}", file=sys.stderr, flush=True)
    x, s = workloads.make(w)
    tree = kifmm.kifmm_tree_build_host(x, w.depth, w.cube[0] + (w.cube[1],))
    ops = kifmm.kifmm_ops_precompute(w.p, eps_pinv=1e-7, eps_svd=1e-6)
    k = kifmm.kifmm_ops_get_info(ops)["rank_m2l"]
    q = torch.from_numpy(s).to(dev)
    pot = torch.empty(w.n, device=dev)
    idx = np.sort(np.random.default_rng(4003).choice(w.n, size=128, replace=False))
    prec = {"workload": w.name, "m2l_rank": k, "forms": {}}
    sample = {"idx": idx}
    for form, fl, passes in (("fp32", 0, 1), ("bf16x3", kifmm.KIFMM_M2L_BF16X3, 3), ("bf16x6", kifmm.KIFMM_M2L_BF16X6, 6)):
        plan = kifmm.kifmm_plan_create(tree, ops, 1, kifmm.KIFMM_POTENTIAL | fl)
        st = kifmm.kifmm_plan_get_stats(plan)
        step = lambda: kifmm.kifmm_evaluate(plan, q, pot, None, stream.cuda_stream)  # noqa: E731
        for _ in range(2):
            step()
        ms = tm.block(step, steps)
        stg = tm.stages(plan, step, max(2, steps // 2))
        peak = PEAK_FP32_TFLOPS if passes == 1 else PEAK_BF16_TFLOPS
        products = st["m2l_stage_pairs"] if passes == 1 else bf16_products(st, passes)
        ach = 2.0 * k * k * products / (stg["m2l"] * 1e-3) / 1e12
        sample[f"phi_{form}"] = pot.cpu().numpy()[idx].astype(np.float64)
        prec["forms"][form] = {"ms_per_evaluate": ms, "mpoints_per_s": w.n / (ms * 1e-3) / 1e6,
                               "m2l_ms": stg["m2l"], "m2l_roofline": {"achieved": ach, "peak": peak,
                                                                      "unit": "TFLOP/s", "frac": ach / peak,
                                                                      "passes": passes},
                               "upper_levels_on_second_stream": bool(st["upper_stream"])}
        kifmm.kifmm_plan_destroy(plan)
        print(f"#   {form}: {ms:.2f} ms/evaluate, M2L {stg['m2l']:.2f} ms ({ach / peak:.3f} of peak)",
              file=sys.stderr, flush=True)
    kifmm.kifmm_ops_destroy(ops)
    kifmm.kifmm_tree_destroy(tree)
    del q, pot, x, s
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "p.npz")
        np.savez(path, **sample)
        acc = run_child("--direct-worker", path, w.name, [], 1)
    if acc:
        prec["rel_l2_vs_direct_sampled"] = acc
        f = prec["forms"]
        prec["speedup_bf16x6_vs_fp32_at_equal_accuracy"] = f["fp32"]["ms_per_evaluate"] / f["bf16x6"]["ms_per_evaluate"]
        prec["speedup_bf16x3_vs_fp32"] = f["fp32"]["ms_per_evaluate"] / f["bf16x3"]["ms_per_evaluate"]
        prec["bf16x6_equal_accuracy"] = acc["bf16x6"] <= 1.25 * acc["fp32"]
    rows["precision"] = prec

    # batching: 4M points on the unit sphere, depth 7, 32 N(0,1) right-hand sides, potentials
    w = workloads.WORKLOADS["sphere4m_p6_d7_r32"]
    print(f"# next: {w.name}", file=sys.stderr, flush=True)
    x, s = workloads.make(w)
    tree = kifmm.kifmm_tree_build_host(x, w.depth, w.cube[0] + (w.cube[1],))
    ops = kifmm.kifmm_ops_precompute(w.p, eps_pinv=1e-7, eps_svd=1e-6)
    k = kifmm.kifmm_ops_get_info(ops)["rank_m2l"]
    q = torch.from_numpy(s).to(dev)
    pot = torch.empty(w.n, 32, device=dev)
    plan = kifmm.kifmm_plan_create(tree, ops, 32, kifmm.KIFMM_POTENTIAL)
    st = kifmm.kifmm_plan_get_stats(plan)
    step = lambda: kifmm.kifmm_evaluate(plan, q, pot, None, stream.cuda_stream)  # noqa: E731
    step()
    ms32 = tm.block(step, max(2, steps // 2))
    stg = tm.stages(plan, step, 2)
    m2l_flop = 2.0 * k * k * st["m2l_pairs"] * 32
    leaf_flop = (9 + 2 * 32) * (st["p2p_pairs"] + w.n * st["n"])
    idx = np.sort(np.random.default_rng(4004).choice(w.n, size=64, replace=False))
    sample = {"idx": idx, "phi_r32": pot.cpu().numpy()[idx].astype(np.float64)}
    kifmm.kifmm_plan_destroy(plan)
    q1 = q[:, 0].contiguous()
    pot1 = torch.empty(w.n, device=dev)
    plan1 = kifmm.kifmm_plan_create(tree, ops, 1, kifmm.KIFMM_POTENTIAL)
    st1 = kifmm.kifmm_plan_get_stats(plan1)
    step1 = lambda: kifmm.kifmm_evaluate(plan1, q1, pot1, None, stream.cuda_stream)  # noqa: E731
    for _ in range(2):
        step1()
    ms1 = tm.block(step1, steps)
    stg1 = tm.stages(plan1, step1, max(2, steps // 2))
    kifmm.kifmm_plan_destroy(plan1)
    kifmm.kifmm_ops_destroy(ops)
    kifmm.kifmm_tree_destroy(tree)
    del q, pot, q1, pot1, x, s
    bat = {"workload": w.name, "m2l_rank": k, "ms_per_evaluate": ms32,
           "point_rhs_per_s": w.n * 32 / (ms32 * 1e-3), "stages_ms": stg,
           "m2l_roofline": {"kernel": "k_m2l_wide", "achieved": m2l_flop / (stg["m2l"] * 1e-3) / 1e12,
                            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"},
           "leaf": {"kernel": "k_leaf_r32", "achieved": leaf_flop / (stg["p2p"] * 1e-3) / 1e12,
                    "flop_per_pair": 9 + 2 * 32, "unit": "TFLOP/s"},
           "one_rhs": {"ms_per_evaluate": ms1, "stages_ms": stg1,
                       "leaf_kernel": "k_leaf_queue" if st1["leaf_queue"] else "k_p2p",
                       "m2l_form": ["blocked", "gathered"][st1["m2l_form"]] if st1["m2l_form"] < 2 else st1["m2l_form"]},
           "batching_speedup": 32 * ms1 / ms32}
    bat["m2l_roofline"]["frac"] = bat["m2l_roofline"]["achieved"] / PEAK_FP32_TFLOPS
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "b.npz")
        np.savez(path, **sample)
        acc = run_child("--direct-worker", path, w.name, [], 1)
    if acc:
        bat["rel_l2_vs_direct_sampled"] = acc["r32"]
        bat["direct_sample_targets"] = acc["targets"]
    print(f"#   32 RHS: {ms32:.1f} ms; one RHS {ms1:.2f} ms; speedup {bat['batching_speedup']:.2f}",
          file=sys.stderr, flush=True)
    rows["batching"] = bat

    # differentiation: 2M points, p = 7, depth 6, forward (potentials and field) + backward
    w = workloads.WORKLOADS["cube2m_p7_d6"]
    print(f"# next: {w.name}", file=sys.stderr, flush=True)
    x, s = workloads.make(w)
    wts = workloads.charges("normal", w.n, w.seed + 2000)
    tree = kifmm.kifmm_tree_build_host(x, w.depth, w.cube[0] + (w.cube[1],))
    ops = kifmm.kifmm_ops_precompute(w.p, eps_pinv=1e-7, eps_svd=1e-6)
    plan = kifmm.kifmm_plan_create(tree, ops, 1, kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT | kifmm.KIFMM_VJP)
    q, wd = torch.from_numpy(s).to(dev), torch.from_numpy(wts).to(dev)
    pot = torch.empty(w.n, device=dev)
    field = torch.empty(w.n, 3, device=dev)
    gc = torch.empty(w.n, device=dev)
    gp = torch.empty(w.n, 3, device=dev)
    fwd = lambda: kifmm.kifmm_evaluate(plan, q, pot, field, stream.cuda_stream)  # noqa: E731

    def fwd_bwd():
        fwd()
        kifmm.kifmm_evaluate_vjp(plan, q, wd, field, gc, gp, stream.cuda_stream)
    for _ in range(2):
        fwd_bwd()
    ms_f = tm.block(fwd, steps)
    ms_fb = tm.block(fwd_bwd, steps)
    idx = np.sort(np.random.default_rng(4005).choice(w.n, size=64, replace=False))
    sample = {"idx": idx, "weights": wts, "phi": pot.cpu().numpy()[idx].astype(np.float64),
              "grad_charges": gc.cpu().numpy()[idx].astype(np.float64),
              "grad_points": gp.cpu().numpy()[idx].astype(np.float64)}
    kifmm.kifmm_plan_destroy(plan)
    kifmm.kifmm_ops_destroy(ops)
    kifmm.kifmm_tree_destroy(tree)
    diff = {"workload": w.name, "forward_ms": ms_f, "forward_backward_ms": ms_fb,
            "forward_mpoints_per_s": w.n / (ms_f * 1e-3) / 1e6,
            "forward_backward_mpoints_per_s": w.n / (ms_fb * 1e-3) / 1e6}
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "d.npz")
        np.savez(path, **sample)
        acc = run_child("--direct-worker", path, w.name, [], 1)
    if acc:
        diff["rel_l2_vs_direct_sampled"] = acc
    print(f"#   forward {ms_f:.2f} ms, forward + backward {ms_fb:.2f} ms", file=sys.stderr, flush=True)
    rows["differentiation"] = diff
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5, help="blocks of --steps evaluates for the mean and spread")
    ap.add_argument("--workload", default="cube1m_p6_d5")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (parity still checked)")
    ap.add_argument("--no-parity", action="store_true",
                    help="profiling runs: no oracle or direct-sum legs; value is null (accuracy not shown)")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the precision, batching and differentiation workloads")
    ap.add_argument("--next-steps", type=int, default=10)
    ap.add_argument("--serial", action="store_true",
                    help="run every kernel on one stream (no ULI overlap with the far field)")
    ap.add_argument("--m2l", choices=["fp32", "bf16x3", "bf16x6"], default="fp32",
                    help="M2L arithmetic: plain FP32, or split bfloat16 (3 or 6 matrix-core passes, FP32 accumulation)")
    ap.add_argument("--backward", action="store_true",
                    help="time forward + backward: evaluate (potentials and field) then the vector-Jacobian "
                         "product of L = sum w_i f_i (adjoint evaluate + combination)")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step in a HIP graph (torch.cuda.graph) and time its replays")
    ap.add_argument("--m2l-form", choices=["auto", "blocked", "gathered"], default="auto")
    ap.add_argument("--upper-stream", choices=["auto", "on", "off"], default="auto")
    ap.add_argument("--leaf", choices=["auto", "blocks", "queue"], default="auto",
                    help="one-RHS leaf kernel: per-parent blocks or the persistent work queue")
    ap.add_argument("--leaf-threads", choices=["auto", "256", "320"], default="auto")
    ap.add_argument("--m2l-rank", type=int, default=None,
                    help="M2L compression rank (default: the workload's; 0: singular values above 1e-6 sigma_max)")
    ap.add_argument("--no-compare-rank", action="store_true",
                    help="skip the timing at the default M2L rank of a workload with a rank of its own")
    ap.add_argument("--sample-leaves", type=int, default=3000)
    ap.add_argument("--sample-seed", type=int, default=2)
    ap.add_argument("--direct-targets", type=int, default=1024)
    ap.add_argument("--direct-grad-targets", type=int, default=256)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (calibrates HBM byte counters) and exit")
    ap.add_argument("--oracle-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--direct-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--timing-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--gpu-sample", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.oracle_worker:
        oracle_worker(args)
        return
    if args.direct_worker:
        direct_worker(args)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe * (1 << 20) // 4, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the evaluate runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design, not built)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_19243_amd import kifmm, workloads

    w = workloads.WORKLOADS[args.workload]
    print(f"# bench {w.name}: n={w.n} depth={w.depth} p={w.p} grad={w.gradient}", file=sys.stderr, flush=True)
    x, s = workloads.make(w)
    cube = w.cube[0] + (w.cube[1],)
    t_setup = time.perf_counter()
    passes = {"fp32": 0, "bf16x3": 3, "bf16x6": 6}[args.m2l]
    bf16 = passes > 0
    m2l_flag = {"fp32": 0, "bf16x3": kifmm.KIFMM_M2L_BF16X3, "bf16x6": kifmm.KIFMM_M2L_BF16X6}[args.m2l]
    R = w.nrhs
    if R > 1:
        if args.backward:
            raise SystemExit("--backward needs a one-RHS workload")
        flags = kifmm.KIFMM_POTENTIAL
    else:
        flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT | (kifmm.KIFMM_SERIAL if args.serial else 0)
        flags |= kifmm.KIFMM_VJP if args.backward else 0
        flags |= {"auto": 0, "blocks": kifmm.KIFMM_LEAF_BLOCKS, "queue": kifmm.KIFMM_LEAF_QUEUE}[args.leaf]
        flags |= {"auto": 0, "256": kifmm.KIFMM_LEAF_THREADS_256, "320": kifmm.KIFMM_LEAF_THREADS_320}[args.leaf_threads]
    m2l_flag |= {"auto": 0, "blocked": kifmm.KIFMM_M2L_BLOCKED, "gathered": kifmm.KIFMM_M2L_GATHER}[args.m2l_form]
    m2l_flag |= {"auto": 0, "on": kifmm.KIFMM_UPPER_STREAM, "off": kifmm.KIFMM_NO_UPPER_STREAM}[args.upper_stream]
    rank = w.m2l_rank if args.m2l_rank is None else args.m2l_rank
    f = kifmm.FMM(x, w.depth, w.p, cube=cube, eps_pinv=1e-7, eps_svd=1e-6, rank=rank, flags=flags | m2l_flag, nrhs=R)
    t_setup = time.perf_counter() - t_setup
    info = kifmm.kifmm_ops_get_info(f.ops)
    stats = kifmm.kifmm_plan_get_stats(f.plan)
    k, n = info["rank_m2l"], info["n_surface"]
    print(f"# setup {t_setup:.1f} s, k={k}, n={n}, stats={stats}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    charges = torch.from_numpy(s).to(dev)
    pot = torch.empty(w.n, device=dev) if R == 1 else torch.empty(w.n, R, device=dev)
    grad = torch.empty(w.n, 3, device=dev) if (R == 1 and (w.gradient or args.backward)) else None
    if args.graph:
        # graphs are captured on a (default-priority) stream of our own, not the null stream
        torch.cuda.synchronize()
        torch.cuda.set_stream(torch.cuda.Stream())
    stream = torch.cuda.current_stream()
    tm = Timer(torch, stream)
    if args.backward:
        weights = torch.from_numpy(workloads.charges("normal", w.n, w.seed + 2000)).to(dev)
        grad_charges = torch.empty(w.n, device=dev)
        grad_points = torch.empty(w.n, 3, device=dev)

    def step_of(plan):
        def step():
            kifmm.kifmm_evaluate(plan, charges, pot, grad, stream.cuda_stream)
            if args.backward:
                kifmm.kifmm_evaluate_vjp(plan, charges, weights, grad, grad_charges, grad_points, stream.cuda_stream)
        return step

    step = step_of(f.plan)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            step()
        torch.cuda.synchronize()
        timed_step = graph.replay
    else:
        timed_step = step
    # the timed region: exactly --steps steps, stage events off; then more blocks for the spread
    blocks = [tm.block(timed_step, args.steps)]
    for _ in range(max(0, args.repeats - 1)):
        blocks.append(tm.block(timed_step, args.steps))
    ms = blocks[0]
    mean_ms, std_ms = mean_std(blocks)
    rates = [w.n / (b * 1e-3) / 1e6 for b in blocks]
    print(f"# {w.name}: {ms:.3f} ms/step (blocks: " + ", ".join(f"{b:.3f}" for b in blocks) + ")",
          file=sys.stderr, flush=True)
    # outputs of the timed evaluates, for the accuracy gate
    phi_all = pot.cpu().numpy()
    grad_all = grad.cpu().numpy() if grad is not None else None
    del graph
    stages = tm.stages(f.plan, step, args.steps)
    print("# stages (ms/call): " + ", ".join(f"{k_}={v:.3f}" for k_, v in stages.items()), file=sys.stderr, flush=True)

    default_rank = None
    extra_phi = {}
    direct_idx = np.sort(np.random.default_rng(4000 + 2).choice(w.n, size=min(args.direct_targets, w.n),
                                                                 replace=False))
    if w.m2l_rank and args.m2l_rank is None and not args.no_compare_rank:
        # the same evaluate with the M2L rank of the 1e-6 singular-value threshold
        fr = kifmm.FMM(x, w.depth, w.p, cube=cube, eps_pinv=1e-7, eps_svd=1e-6, rank=0, flags=flags | m2l_flag,
                       nrhs=R)
        kr = kifmm.kifmm_ops_get_info(fr.ops)["rank_m2l"]
        stepr = step_of(fr.plan)
        for _ in range(args.warmup):
            stepr()
        msr = tm.block(stepr, args.steps)
        stagesr = tm.stages(fr.plan, stepr, args.steps)
        extra_phi["extra_phi_default_rank"] = pot.cpu().numpy()[direct_idx].astype(np.float64)
        fr.close()
        default_rank = {"m2l_rank": kr, "ms_per_step": msr, "value": w.n / (msr * 1e-3) / 1e6,
                        "m2l_ms": stagesr["m2l"], "stages_ms": stagesr}
        print(f"# rank {kr}: {msr:.3f} ms/step", file=sys.stderr, flush=True)

    # The U-list kernel of the default layout shares the GPU with the far field, so its span says
    # little about its own speed: the fused D2T + ULI kernel of a one-stream plan on the same tree
    # and operators, with the main plan's leaf kernel and workgroup size, is timed alone.
    p2p_alone = None
    if R == 1 and not args.serial and not args.graph:
        layout = kifmm.KIFMM_UPPER_STREAM | kifmm.KIFMM_NO_UPPER_STREAM
        pin = kifmm.KIFMM_LEAF_QUEUE if stats["leaf_queue"] else (
            kifmm.KIFMM_LEAF_BLOCKS | (kifmm.KIFMM_LEAF_THREADS_256 if stats["p2p_threads"] == 256
                                       else kifmm.KIFMM_LEAF_THREADS_320))
        fl_s = (flags & ~(kifmm.KIFMM_VJP | kifmm.KIFMM_LEAF_QUEUE | kifmm.KIFMM_LEAF_BLOCKS |
                          kifmm.KIFMM_LEAF_THREADS_256 | kifmm.KIFMM_LEAF_THREADS_320))
        plan_s = kifmm.kifmm_plan_create(f.tree, f.ops, 1, fl_s | (m2l_flag & ~layout) | kifmm.KIFMM_SERIAL | pin)
        st_s = kifmm.kifmm_plan_get_stats(plan_s)
        steps_ = lambda: kifmm.kifmm_evaluate(plan_s, charges, pot, grad, stream.cuda_stream)  # noqa: E731
        for _ in range(2):
            steps_()
        stg_s = tm.stages(plan_s, steps_, 10)
        kifmm.kifmm_plan_destroy(plan_s)
        ms_s = stg_s["p2p"]
        pairs_s = stats["p2p_pairs"] + w.n * n * (1 if w.depth >= 2 else 0)
        fpp = P2P_FLOPS_PER_PAIR if grad is not None else 9 + 2 * R
        tf_s = fpp * pairs_s / (ms_s * 1e-3) / 1e12
        p2p_alone = {"kernel": leaf_kernel_name(st_s, True, 1) + " (fused D2T + ULI, one-stream plan, alone on the GPU)",
                     "bound": "alu", "achieved": tf_s, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf_s / PEAK_FP32_TFLOPS, "ms_per_launch": ms_s, "pairs_per_launch": pairs_s,
                     "flop_per_pair": fpp, "launches": 10, "p2p_threads": st_s["p2p_threads"],
                     "leaf_queue": bool(st_s["leaf_queue"])}
        print(f"# fused D2T + ULI alone: {ms_s:.3f} ms, {tf_s:.1f} TFLOP/s", file=sys.stderr, flush=True)

    # M2L (dominant kernel): 2 k^2 FLOP per (target, source) V-list pair; the split-bfloat16
    # forms execute each product as 3 or 6 bfloat16 products, counted against the BF16 peak.
    m2l_ms = stages["m2l"]
    m2l_flop = 2.0 * k * k * stats["m2l_stage_pairs"] * R
    m2l_tflops = m2l_flop / (m2l_ms * 1e-3) / 1e12
    bf16_flop = bf16_products(stats, passes) * 2.0 * k * k * R
    m2l_kernel = (f"k_m2l_bf16<{passes // 3 + 1}, 0>" if bf16 else
                  ["k_m2l<0>", "k_m2l_gather<0>", "k_m2l_wide", "k_m2l_bf16"][stats["m2l_form"]])
    traffic = load_traffic(w.name, m2l_kernel, {"m2l_rank": k, "upper_levels_on_second_stream": bool(stats["upper_stream"])})
    p2p_ms = stages["p2p"]
    fused = args.serial or R > 1 or w.depth < 2   # one leaf kernel does D2T and ULI
    flop_pair = P2P_FLOPS_PER_PAIR if grad is not None else 9 + 2 * R
    d2t_pairs = w.n * n * (1 if w.depth >= 2 else 0)
    p2p_pairs = stats["p2p_pairs"] + (d2t_pairs if fused else 0)
    p2p_tflops = flop_pair * p2p_pairs / (p2p_ms * 1e-3) / 1e12
    if bf16:
        ach = bf16_flop / (m2l_ms * 1e-3) / 1e12
        roofline = {"kernel": m2l_kernel, "bound": "mfma", "achieved": ach,
                    "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_BF16_TFLOPS,
                    "traffic": traffic, "passes": passes, "fp32_equivalent_tflops": m2l_tflops}
    else:
        roofline = {"kernel": m2l_kernel, "bound": "mfma", "achieved": m2l_tflops, "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": m2l_tflops / PEAK_FP32_TFLOPS, "traffic": traffic}
    roofline.update({"ms_per_launch": m2l_ms, "algorithmic_flop_per_launch": m2l_flop,
                     "v_list_pairs": stats["m2l_stage_pairs"], "v_list_pairs_all_levels": stats["m2l_pairs"]})

    result = {
        "metric": METRIC,
        "value": w.n / (ms * 1e-3) / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"f32, M2L {args.m2l} (f32 accumulation)" if bf16 else "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_points": w.n, "distribution": w.distribution, "charges": w.charges,
                   "p": w.p, "n_surface": n, "m2l_rank": k, "depth": w.depth, "nrhs": w.nrhs,
                   "outputs": "potential+gradient" if w.gradient else "potential", "parallelism": "single-gpu",
                   "uli_overlap": not args.serial, "m2l": args.m2l, "hip_graph": args.graph,
                   "m2l_form": ["blocked", "gathered", "wide (32 right-hand sides)", "split bfloat16 blocked"][
                       stats["m2l_form"]],
                   "upper_levels_on_second_stream": bool(stats["upper_stream"]),
                   "m2l_lds_slab": stats["m2l_lds_slab"],
                   "leaf_kernel": leaf_kernel_name(stats, args.serial, R),
                   "p2p_threads_per_workgroup": stats["p2p_threads"],
                   "step": ("forward (potentials and field) + backward (vector-Jacobian product of "
                            "sum w_i f_i, w ~ N(0,1))") if args.backward else "evaluate"},
        "repeats": {"blocks": len(blocks), "steps_per_block": args.steps, "ms_per_step": blocks,
                    "mean_ms": mean_ms, "std_ms": std_ms, "mean_mpoints_per_s": mean_std(rates)[0],
                    "std_mpoints_per_s": mean_std(rates)[1]},
        "roofline": roofline,
        "p2p": {"kernel": leaf_kernel_name(stats, args.serial, R) + ("" if args.serial or R > 1 else
                                                                      " (ULI, beside the far field)"),
                "bound": "alu", "achieved": p2p_tflops, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": p2p_tflops / PEAK_FP32_TFLOPS, "ms_per_launch": p2p_ms,
                "pairs_per_launch": p2p_pairs, "flop_per_pair": flop_pair,
                "d2t_ms_per_launch": stages["l2p"] if stages["l2p"] > 0 else None, "d2t_pairs_per_launch": d2t_pairs},
        "p2p_alone": p2p_alone,
        "stages_ms": stages,
        "plan_tuning_us": {key: v for key, v in stats.items() if key.startswith("tune_us_") and v},
        "setup_s": t_setup,
        "cpu_baseline": None,
    }
    if default_rank is not None:
        result["default_rank"] = default_rank
    if R > 1:
        result["point_rhs_per_s"] = w.n * R / (ms * 1e-3)
    f.close()
    del charges, pot, grad

    # further workloads (GPU), before the CPU legs so that those time an idle host
    if not args.no_next and args.workload == "cube1m_p6_d5" and not (bf16 or args.backward or args.graph or args.serial):
        result["next_rows"] = next_rows(args, torch, dev)

    # The oracle leg (a child process with single-threaded BLAS): the oracle timed on a sample,
    # the GPU's parity with it on the sampled leaves, and the direct sum at sampled targets;
    # then the same timing with every core the process may use.
    gate = {"oracle_tol": ORACLE_TOL[args.m2l], "direct_tol": DIRECT_TOL}
    if args.no_parity:
        gate.update(passed=False, reason="not checked (--no-parity)")
        result.update(value=None, accuracy_gate=gate)
        print(json.dumps(result), flush=True)
        return
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "gpu.npz")
        sample = {"phi": phi_all.astype(np.float64), "direct_idx": direct_idx}
        if grad_all is not None:
            sample["grad"] = grad_all.astype(np.float64)
        sample.update(extra_phi)
        np.savez(path, **sample)
        print("# oracle leg (1 thread)...", file=sys.stderr, flush=True)
        base = ["--sample-leaves", str(args.sample_leaves), "--sample-seed", str(args.sample_seed),
                "--m2l-rank", str(rank), "--direct-grad-targets", str(args.direct_grad_targets)]
        one = run_child("--oracle-worker", path, w.name, base, 1)
        cores = len(os.sched_getaffinity(0))
        allc = None
        if one is not None and not args.no_cpu_baseline:
            print(f"# oracle leg ({cores} threads)...", file=sys.stderr, flush=True)
            allc = run_child("--oracle-worker", path, w.name, base + ["--timing-only"], cores)
    if one is not None:
        result["accuracy"] = {"oracle_parity": one["oracle_parity"], "direct": one["direct"]}
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = one["timing"]
            if allc is not None:
                result["cpu_baseline_all_cores"] = allc["timing"]
        op, dr = one["oracle_parity"], one["direct"]
        checks = [op["rel_l2_phi"] <= gate["oracle_tol"], dr["rel_l2_phi"] <= DIRECT_TOL]
        if "rel_l2_grad" in op:
            checks.append(op["rel_l2_grad"] <= gate["oracle_tol"])
        gate["passed"] = all(checks)
        if default_rank is not None and "phi_default_rank" in dr:
            default_rank["rel_l2_vs_direct_sampled"] = dr["phi_default_rank"]
    else:
        gate["passed"] = False
        gate["reason"] = "the oracle leg did not run or failed"
    result["accuracy_gate"] = gate
    if not gate["passed"]:
        result["value"] = None
    print(json.dumps(result), flush=True)
    if not gate["passed"]:
        sys.exit(1)


if __name__ == "__main__":
    main()
