#!/usr/bin/env python3
"""Throughput of one kiFMM evaluate (3D Laplace) on one MI355X.

A step is one full evaluate through the C ABI: permute, S2U (P2M), U2U, M2L
compression and VLI, post + D2D, fused D2T + ULI (L2P + P2P) writing potentials
and gradients in input order.  Inputs are resident in HBM before timing; tree
build and operator precompute are setup and are not timed.

Prints one JSON line: metric/value (Mpoints/s = N / time per evaluate), the
roofline of the dominant kernel (M2L, FP32 matrix cores) measured with HIP
events on the evaluate stream, the P2P kernel's FLOP rate (overlapped with the far
field, and alone in a one-stream plan), and the FP64 oracle
timed on a bounded sample on the host CPU.

`--m2l bf16x3` runs M2L as three bfloat16 matrix-core passes with FP32
accumulation (roofline against the BF16 peak, three passes counted);
`--compare-fp32` then also times the plain FP32 form on the same tree and
operators and reports both forms' accuracy against the direct sum.
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


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2604_19243_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload, kernel, config):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None if stale, missing
    or measured on another launch configuration (M2L rank, second stream)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            entries = json.load(f)[kernel][workload]
    except (OSError, KeyError, ValueError):
        return None
    for entry in entries if isinstance(entries, list) else [entries]:
        if entry.get("kernels_hip_sha256_16") == kernel_source_hash() and entry.get("config") == config:
            return float(entry["hbm_bytes_per_launch"])
    return None


def cpu_baseline_worker(args):
    """Runs in a child process with single-threaded BLAS: times the FP64 oracle on a sample."""
    import numpy as np

    from oracle import direct, fmm, operators, tree
    from paper_2604_19243_amd import workloads

    w = workloads.WORKLOADS[args.workload]
    x32, s32 = workloads.make(w)
    x, s = x32.astype(np.float64), s32.astype(np.float64)

    # accuracy of the GPU run(s): oracle direct sum at sampled targets, in blocks of sources
    gpu = np.load(args.gpu_sample)
    idx = gpu["idx"]
    ref = np.zeros((len(idx),) + s.shape[1:])
    for a in range(0, len(x), 250_000):
        ref += direct.potential(x[idx], x[a:a + 250_000], s[a:a + 250_000])
    acc = {"rel_l2_vs_direct_sampled": direct.rel_l2(gpu["phi"], ref), "direct_sample_targets": int(len(idx))}
    if "phi_fp32" in gpu:
        acc["fp32_rel_l2_vs_direct_sampled"] = direct.rel_l2(gpu["phi_fp32"], ref)
    if "phi_rank" in gpu:
        acc["rank_rel_l2_vs_direct_sampled"] = direct.rel_l2(gpu["phi_rank"], ref)
    if args.accuracy_only:
        print(json.dumps(acc), flush=True)
        return

    c, r = w.cube
    t = tree.Tree(x, w.depth, c, r)
    rank = w.m2l_rank if args.m2l_rank is None else args.m2l_rank
    ops = operators.Operators(w.p, eps_pinv=1e-7, m2l="compressed", eps_svd=1e-6, rank=rank or None)
    L = w.depth
    for l in range(2, L + 1):
        ops.compression(t.radius(l))          # operator setup, not timed (as on the GPU)
    s2 = s[:, None]
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
    phi, _ = fmm.leaf_pass(t, ops, s2, d, leaves, w.gradient)
    t3 = time.perf_counter()
    boxes_all = sum(len(t.boxes[l]) for l in range(2, L + 1))
    boxes_sampled = sum(len(needed[l]) for l in range(2, L + 1))
    t_full = (t1 - t0) + (t2 - t1) * boxes_all / boxes_sampled + (t3 - t2) * len(all_leaves) / len(leaves)

    out = {
        "value": w.n / t_full / 1e6, "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle, single thread: full upward pass ({t1 - t0:.2f} s) timed; downward pass "
                   f"timed on the {boxes_sampled} ancestors of {len(leaves)} random leaves ({t2 - t1:.2f} s) and "
                   f"leaf pass on those leaves ({t3 - t2:.2f} s), each scaled by box/leaf counts to the full "
                   f"workload; extrapolated evaluate {t_full:.1f} s"),
        "seconds_measured": t3 - t0, "seconds_extrapolated": t_full,
    }
    out.update(acc)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube1m_p6_d5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="run every kernel on one stream (no ULI overlap with the far field)")
    ap.add_argument("--m2l", choices=["fp32", "bf16x3", "bf16x6"], default="fp32",
                    help="M2L arithmetic: plain FP32, or split bfloat16 (3 or 6 matrix-core passes, FP32 accumulation)")
    ap.add_argument("--compare-fp32", action="store_true",
                    help="with a split-bfloat16 --m2l: also time the plain FP32 form on the same tree and operators")
    ap.add_argument("--backward", action="store_true",
                    help="time forward + backward: evaluate (potentials and field) then the vector-Jacobian "
                         "product of L = sum w_i f_i (adjoint evaluate + combination)")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step in a HIP graph (torch.cuda.graph) and time its replays")
    ap.add_argument("--m2l-form", choices=["auto", "blocked", "gathered"], default="auto",
                    help="one-RHS FP32 M2L form (auto: the faster, timed at plan creation)")
    ap.add_argument("--upper-stream", choices=["auto", "on", "off"], default="auto",
                    help="levels above the leaves on the plan's second stream (auto: timed at plan creation)")
    ap.add_argument("--m2l-rank", type=int, default=None,
                    help="M2L compression rank (default: the workload's; 0: singular values above 1e-6 sigma_max)")
    ap.add_argument("--no-compare-rank", action="store_true",
                    help="skip the second timing, at the default M2L rank, of a workload with a rank of its own")
    ap.add_argument("--compare-single", action="store_true",
                    help="with a multi-RHS workload: also time a one-RHS plan on the same tree and operators")
    ap.add_argument("--sample-leaves", type=int, default=3000)
    ap.add_argument("--sample-seed", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (calibrates HBM byte counters) and exit")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--accuracy-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--gpu-sample", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args)
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
        # several right-hand sides: potentials, one stream
        if args.backward:
            raise SystemExit("--backward needs a one-RHS workload")
        flags = kifmm.KIFMM_POTENTIAL
    else:
        flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT | (kifmm.KIFMM_SERIAL if args.serial else 0)
        flags |= kifmm.KIFMM_VJP if args.backward else 0
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
    if args.backward:
        weights = torch.from_numpy(workloads.charges("normal", w.n, w.seed + 2000)).to(dev)
        grad_charges = torch.empty(w.n, device=dev)
        grad_points = torch.empty(w.n, 3, device=dev)

    io = {"charges": charges, "pot": pot}

    def step(plan):
        kifmm.kifmm_evaluate(plan, io["charges"], io["pot"], grad, stream.cuda_stream)
        if args.backward:
            kifmm.kifmm_evaluate_vjp(plan, charges, weights, grad, grad_charges, grad_points, stream.cuda_stream)

    def timed(plan, label):
        """Warm-up, then exactly args.steps steps between two events on the evaluate stream."""
        for _ in range(args.warmup):
            step(plan)
        torch.cuda.synchronize()
        if args.graph:
            # one step captured on the evaluate stream; the timed region replays it
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                step(plan)
            torch.cuda.synchronize()
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(args.steps):
                g.replay()
            end.record(stream)
            torch.cuda.synchronize()
            ms_ = start.elapsed_time(end) / args.steps
            print(f"# {label} (graph replay): {ms_:.3f} ms/step", file=sys.stderr, flush=True)
            del g
            kifmm.kifmm_plan_set_timing(plan, True)
            kifmm.kifmm_plan_get_stage_times(plan, reset=True)
            step(plan)  # one eager step for the stage breakdown
            torch.cuda.synchronize()
            st = kifmm.kifmm_plan_get_stage_times(plan, reset=True)
            kifmm.kifmm_plan_set_timing(plan, False)
            return ms_, {k_: v[0] / max(v[1], 1) for k_, v in st.items()}
        kifmm.kifmm_plan_set_timing(plan, True)
        kifmm.kifmm_plan_get_stage_times(plan, reset=True)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            step(plan)
        end.record(stream)
        torch.cuda.synchronize()
        ms_ = start.elapsed_time(end) / args.steps
        st = kifmm.kifmm_plan_get_stage_times(plan, reset=True)
        kifmm.kifmm_plan_set_timing(plan, False)
        print(f"# {label}: {ms_:.3f} ms/evaluate; stages (ms/call): "
              + ", ".join(f"{k_}={v[0] / max(v[1], 1):.3f}" for k_, v in st.items()), file=sys.stderr, flush=True)
        return ms_, {k_: v[0] / max(v[1], 1) for k_, v in st.items()}

    idx = np.sort(np.random.default_rng(4002).choice(w.n, size=min(256, w.n), replace=False))
    ms, stages = timed(f.plan, "m2l " + args.m2l)
    phi_sample = pot.cpu().numpy()[idx].astype(np.float64)
    fp32_form = None
    single = None
    if R > 1 and args.compare_single:
        plan1 = kifmm.kifmm_plan_create(f.tree, f.ops, 1, kifmm.KIFMM_POTENTIAL | m2l_flag)
        io.update(charges=charges[:, 0].contiguous(), pot=torch.empty(w.n, device=dev))
        ms1, stages1 = timed(plan1, "one right-hand side")
        kifmm.kifmm_plan_destroy(plan1)
        io.update(charges=charges, pot=pot)
        single = {"ms_per_evaluate": ms1, "stages_ms": stages1, "batching_speedup": R * ms1 / ms}
    if bf16 and args.compare_fp32:
        plan32 = kifmm.kifmm_plan_create(f.tree, f.ops, R, flags)
        ms32, stages32 = timed(plan32, "m2l fp32")
        phi32_sample = pot.cpu().numpy()[idx].astype(np.float64)
        kifmm.kifmm_plan_destroy(plan32)
        fp32_form = {"ms_per_step": ms32, "m2l_ms": stages32["m2l"], "stages_ms": stages32,
                     "speedup_evaluate": ms32 / ms, "speedup_m2l": stages32["m2l"] / stages["m2l"]}

    default_rank = None
    phir_sample = None
    if w.m2l_rank and args.m2l_rank is None and not args.no_compare_rank:
        # the same evaluate with the M2L rank of the 1e-6 singular-value threshold
        fr = kifmm.FMM(x, w.depth, w.p, cube=cube, eps_pinv=1e-7, eps_svd=1e-6, rank=0, flags=flags | m2l_flag,
                       nrhs=R)
        kr = kifmm.kifmm_ops_get_info(fr.ops)["rank_m2l"]
        msr, stagesr = timed(fr.plan, f"m2l {args.m2l}, rank {kr}")
        phir_sample = pot.cpu().numpy()[idx].astype(np.float64)
        fr.close()
        default_rank = {"m2l_rank": kr, "ms_per_step": msr, "value": w.n / (msr * 1e-3) / 1e6,
                        "m2l_ms": stagesr["m2l"], "stages_ms": stagesr}

    # The ULI kernel of the default layout shares the GPU with the far field, so its span says
    # little about its own speed: the fused D2T + ULI kernel of a one-stream plan on the same
    # tree and operators is timed alone (stage events on the evaluate stream).
    p2p_alone = None
    if R == 1 and not args.serial and not args.graph:
        layout = kifmm.KIFMM_UPPER_STREAM | kifmm.KIFMM_NO_UPPER_STREAM
        plan_s = kifmm.kifmm_plan_create(f.tree, f.ops, 1, (flags & ~kifmm.KIFMM_VJP) | (m2l_flag & ~layout)
                                         | kifmm.KIFMM_SERIAL)
        for _ in range(2):
            kifmm.kifmm_evaluate(plan_s, charges, pot, grad, stream.cuda_stream)
        torch.cuda.synchronize()
        kifmm.kifmm_plan_set_timing(plan_s, True)
        kifmm.kifmm_plan_get_stage_times(plan_s, reset=True)
        for _ in range(10):
            kifmm.kifmm_evaluate(plan_s, charges, pot, grad, stream.cuda_stream)
        torch.cuda.synchronize()
        st_s = kifmm.kifmm_plan_get_stage_times(plan_s, reset=True)
        kifmm.kifmm_plan_destroy(plan_s)
        ms_s = st_s["p2p"][0] / max(st_s["p2p"][1], 1)
        pairs_s = stats["p2p_pairs"] + w.n * n * (1 if w.depth >= 2 else 0)
        fpp = P2P_FLOPS_PER_PAIR if grad is not None else 9 + 2 * R
        tf_s = fpp * pairs_s / (ms_s * 1e-3) / 1e12
        p2p_alone = {"kernel": "k_p2p<0> (fused D2T + ULI, one-stream plan, alone on the GPU)", "bound": "alu",
                     "achieved": tf_s, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": tf_s / PEAK_FP32_TFLOPS,
                     "ms_per_launch": ms_s, "pairs_per_launch": pairs_s, "flop_per_pair": fpp, "launches": 10}
        print(f"# fused D2T + ULI alone: {ms_s:.3f} ms, {tf_s:.1f} TFLOP/s", file=sys.stderr, flush=True)

    # M2L (dominant kernel): 2 k^2 FLOP per (target, source) V-list pair; the split-bfloat16
    # forms execute each product as 3 or 6 bfloat16 products, counted against the BF16 peak.
    m2l_ms = stages["m2l"]
    # the pairs of the KIFMM_STAGE_M2L launch (the leaf level alone when the levels above it
    # run beside it on the plan's second stream)
    m2l_flop = 2.0 * k * k * stats["m2l_stage_pairs"] * R
    m2l_tflops = m2l_flop / (m2l_ms * 1e-3) / 1e12
    # the KIFMM_STAGE_M2L launch (instance 0; the levels above the leaves, when they run on the
    # plan's second stream, are instance 1)
    m2l_kernel = (f"k_m2l_bf16<{passes // 3 + 1}, 0>" if bf16 else
                  ["k_m2l<0>", "k_m2l_gather<0>", "k_m2l_wide", "k_m2l_bf16"][stats["m2l_form"]])
    traffic = load_traffic(w.name, m2l_kernel, {"m2l_rank": k, "upper_levels_on_second_stream": bool(stats["upper_stream"])})
    # Leaf kernels: 20 FLOP per U-list pair (ULI) and per (target, downward-equivalent point) pair (D2T).
    # By default ULI runs on the plan's own stream beside the far field and D2T is a separate
    # kernel; with --serial one fused kernel does both.
    # Potentials only: 9 + 2R FLOP per pair (the geometry once, 2 per right-hand side).
    p2p_ms = stages["p2p"]
    fused = args.serial or R > 1
    flop_pair = P2P_FLOPS_PER_PAIR if grad is not None else 9 + 2 * R
    d2t_pairs = w.n * n * (1 if w.depth >= 2 else 0)
    p2p_pairs = stats["p2p_pairs"] + (d2t_pairs if fused else 0)
    p2p_tflops = flop_pair * p2p_pairs / (p2p_ms * 1e-3) / 1e12
    l2p_ms = stages["l2p"]
    if bf16:
        roofline = {"kernel": m2l_kernel, "bound": "mfma", "achieved": passes * m2l_tflops,
                    "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": passes * m2l_tflops / PEAK_BF16_TFLOPS,
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
                   "p2p_threads_per_workgroup": stats["p2p_threads"],
                   "step": ("forward (potentials and field) + backward (vector-Jacobian product of "
                            "sum w_i f_i, w ~ N(0,1))") if args.backward else "evaluate"},
        "roofline": roofline,
        "p2p": {"kernel": (f"k_leaf_multi<{R}> (fused D2T + ULI)" if R > 1 else
                           "k_p2p<0>" if args.serial else "k_p2p<1> (ULI, overlapped with the far field)"),
                "bound": "alu", "achieved": p2p_tflops, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": p2p_tflops / PEAK_FP32_TFLOPS, "ms_per_launch": p2p_ms,
                "pairs_per_launch": p2p_pairs, "flop_per_pair": flop_pair,
                "d2t_ms_per_launch": None if fused else l2p_ms, "d2t_pairs_per_launch": d2t_pairs},
        "p2p_alone": p2p_alone,
        "stages_ms": stages,
        "setup_s": t_setup,
        "cpu_baseline": None,
    }
    if fp32_form is not None:
        result["fp32_form"] = fp32_form
    if default_rank is not None:
        result["default_rank"] = default_rank
    if R > 1:
        result["point_rhs_per_s"] = w.n * R / (ms * 1e-3)
    if single is not None:
        result["single_rhs"] = single

    # The oracle leg (a child process with single-threaded BLAS): the direct sum at the sampled
    # targets for the accuracy figures and, unless skipped, the oracle timed on a bounded sample.
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "gpu_sample.npz")
        extra = {"phi_fp32": phi32_sample} if fp32_form is not None else {}
        if phir_sample is not None:
            extra["phi_rank"] = phir_sample
        np.savez(path, idx=idx, phi=phi_sample, **extra)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        print("# oracle leg (1 thread)...", file=sys.stderr, flush=True)
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", "--workload", w.name,
               "--sample-leaves", str(args.sample_leaves), "--sample-seed", str(args.sample_seed),
               "--m2l-rank", str(rank), "--gpu-sample", path] + (["--accuracy-only"] if args.no_cpu_baseline else [])
        r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
        if r.returncode == 0:
            cb = json.loads(r.stdout.strip().splitlines()[-1])
            result["rel_l2_vs_direct_sampled"] = cb.pop("rel_l2_vs_direct_sampled")
            result["direct_sample_targets"] = cb.pop("direct_sample_targets")
            if "fp32_rel_l2_vs_direct_sampled" in cb:
                result["fp32_form"]["rel_l2_vs_direct_sampled"] = cb.pop("fp32_rel_l2_vs_direct_sampled")
            if "rank_rel_l2_vs_direct_sampled" in cb:
                result["default_rank"]["rel_l2_vs_direct_sampled"] = cb.pop("rank_rel_l2_vs_direct_sampled")
            if not args.no_cpu_baseline:
                result["cpu_baseline"] = cb
        else:
            print(r.stderr[-2000:], file=sys.stderr, flush=True)
    f.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
