"""The two forms of the plain FP32 M2L for one right-hand side, forced with
KIFMM_M2L_BLOCKED / KIFMM_M2L_GATHER, against the FP64 oracle and against each
other; and the plan's own choice between them (timed at plan creation).

Tolerance: relative L2 <= 1e-6 against the oracle (plain FP32 path).
"""

import numpy as np
import pytest

from gpu_helpers import assert_parity, gpu_evaluate, leaf_groups, log, oracle_evaluate, rel_l2
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6
UNIT = (0.5, 0.5, 0.5, 0.5)
SPHERE = (0.0, 0.0, 0.0, 1.0)


@pytest.mark.parametrize("name,n,depth,p,dist,charges,rank", [
    ("cube20k_p6_d3", 20_000, 3, 6, "cube", "uniform01", 0),
    ("sphere", 30_000, 5, 6, "sphere", "normal", 0),       # sparse: the gathered form's case
    ("ragged", 7_777, 4, 5, "cube", "uniform11", 0),
    ("sparse_deep", 2_000, 6, 4, "cube", "uniform01", 0),
    ("p8", 8_000, 3, 8, "cube", "uniform11", 0),
    ("sphere_rank94", 30_000, 5, 6, "sphere", "normal", 94),  # three 32-row blocks
])
def test_gathered_m2l_parity_with_oracle(name, n, depth, p, dist, charges, rank):
    log(f"gathered M2L parity {name} n={n} depth={depth} p={p} rank={rank}")
    x = workloads.points(dist, n, 1001 if name.startswith("cube20k") else 610 + n)
    s = workloads.charges(charges, n, 2001 if name.startswith("cube20k") else 620 + n)
    cube = UNIT if dist == "cube" else SPHERE
    phi, g, f = gpu_evaluate(x, s, depth, p, cube, m2l="gather", rank=rank)
    assert kifmm.kifmm_plan_get_stats(f.plan)["m2l_form"] == 1
    f.close()
    phb, gb, f = gpu_evaluate(x, s, depth, p, cube, m2l="blocked", rank=rank)
    assert kifmm.kifmm_plan_get_stats(f.plan)["m2l_form"] == 0
    f.close()
    rphi, rg, t, _ = oracle_evaluate(x, s, depth, p, cube, rank=rank or None)
    assert_parity("gathered phi", phi, rphi, leaf_groups(t), TOL)
    assert_parity("gathered grad", g, rg, leaf_groups(t), TOL)
    d = rel_l2(phi, phb)
    log(f"  gathered vs blocked {d:.3e}")
    assert d < TOL


def test_autotuned_form_is_reported_and_correct():
    log("autotuned M2L form")
    w = workloads.WORKLOADS["cube20k_p6_d3"]
    x, s = workloads.make(w)
    c = w.cube[0] + (w.cube[1],)
    phi, g, f = gpu_evaluate(x, s, w.depth, w.p, c)
    form = kifmm.kifmm_plan_get_stats(f.plan)["m2l_form"]
    f.close()
    assert form in (0, 1)
    rphi, rg, t, _ = oracle_evaluate(x, s, w.depth, w.p, c)
    assert_parity(f"phi, chosen form {form}", phi, rphi, leaf_groups(t), TOL)
    assert_parity("grad", g, rg, leaf_groups(t), TOL)


def test_m2l_form_flag_errors():
    x = workloads.points("cube", 400, 58)
    with pytest.raises(kifmm.KifmmError):
        kifmm.FMM(x, 3, 4, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_M2L_BLOCKED | kifmm.KIFMM_M2L_GATHER)
    with pytest.raises(kifmm.KifmmError):
        kifmm.FMM(x, 3, 4, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_M2L_GATHER | kifmm.KIFMM_M2L_BF16X3)
    with pytest.raises(kifmm.KifmmError):
        kifmm.FMM(x, 3, 4, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_M2L_GATHER, nrhs=4)


@pytest.mark.parametrize("rank", [0, 94])
def test_upper_levels_stream_flags(rank):
    # The levels above the leaves on the plan's second stream (forced on) or on the
    # caller's stream (forced off): the same kernels on the same data, so the same bits.
    log(f"upper-level stream on/off rank={rank}")
    x = workloads.points("cube", 40_000, 71)
    s = workloads.charges("uniform11", 40_000, 72)
    out = {}
    for name, fl in (("on", kifmm.KIFMM_UPPER_STREAM), ("off", kifmm.KIFMM_NO_UPPER_STREAM)):
        # no timed choices: both plans take the same LDS slab (which groups the FP32 sums)
        phi, g, f = gpu_evaluate(x, s, 4, 6, UNIT, rank=rank, m2l="blocked", flags=fl | kifmm.KIFMM_NO_AUTOTUNE)
        st = kifmm.kifmm_plan_get_stats(f.plan)
        assert st["upper_stream"] == (1 if name == "on" else 0)
        assert st["p2p_threads"] == 320   # the default without timing
        f.close()
        out[name] = (phi, g)
    np.testing.assert_array_equal(out["on"][0], out["off"][0])
    np.testing.assert_array_equal(out["on"][1], out["off"][1])
    rphi, rg, t, _ = oracle_evaluate(x, s, 4, 6, UNIT, rank=rank or None)
    assert_parity("phi", out["on"][0], rphi, leaf_groups(t), TOL)
    assert_parity("grad", out["on"][1], rg, leaf_groups(t), TOL)


def test_plan_time_choices_are_timed_once_per_shape():
    # The timed choices (M2L form and LDS slab, stream layout, leaf kernel) are kept for the
    # process: a second plan of the same shape takes them without timing and gives the same
    # bits; a plan of another shape times its own.
    log("autotuner cache")
    x = workloads.points("cube", 30_000, 73)
    s = workloads.charges("uniform11", 30_000, 74)
    p1, g1, f1 = gpu_evaluate(x, s, 4, 5, UNIT)
    st1 = kifmm.kifmm_plan_get_stats(f1.plan)
    p2, g2, f2 = gpu_evaluate(x, s, 4, 5, UNIT)
    st2 = kifmm.kifmm_plan_get_stats(f2.plan)
    f1.close()
    f2.close()
    assert st2["tuned_from_cache"] == 1
    for key in ("m2l_form", "m2l_lds_slab", "upper_stream", "p2p_threads", "leaf_queue", "queue_per_cu"):
        assert st1[key] == st2[key], key
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(g1, g2)
    if st1["m2l_form"] == 0:   # the blocked form's slab was timed
        assert sum(st1[f"tune_us_slab_{k}"] > 0 for k in (24, 32, 40, 48)) >= 2
    _, _, f3 = gpu_evaluate(x[:20_000], s[:20_000], 4, 5, UNIT)
    assert kifmm.kifmm_plan_get_stats(f3.plan)["tuned_from_cache"] == 0
    f3.close()
