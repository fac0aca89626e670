"""kifmm_evaluate_vjp_noalloc (its two fields in the library's static device array)
against kifmm_evaluate_vjp (its fields in plan memory), through the C ABI.

Both run the same kernels in the same order on the same inputs, so the results must
agree bit for bit; the oracle's parity of kifmm_evaluate_vjp is tested in
test_gpu_vjp.py.  Two calls in a row, the second with a smaller input (the array keeps
the first call's contents), and the size limit.
"""

import numpy as np
import pytest

from gpu_helpers import log
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

UNIT = (0.5, 0.5, 0.5, 0.5)


def _both(n, depth, p, seed, with_field):
    import torch
    x = workloads.points("cube", n, seed)
    s = workloads.charges("uniform11", n, seed + 1)
    w = workloads.charges("normal", n, seed + 2)
    flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT
    f_ref = kifmm.FMM(x, depth, p, cube=UNIT, flags=flags | kifmm.KIFMM_VJP)
    f_na = kifmm.FMM(x, depth, p, cube=UNIT, flags=flags | kifmm.KIFMM_LEAF_BLOCKS | kifmm.KIFMM_NO_UPPER_STREAM)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    sd, wd = torch.from_numpy(s).to(dev), torch.from_numpy(w).to(dev)
    field = None
    if with_field:
        field = torch.empty(n, 3, device=dev)
        kifmm.kifmm_evaluate(f_ref.plan, sd, None, field, stream)
    out = {}
    for label, f, fn in (("plan", f_ref, kifmm.kifmm_evaluate_vjp), ("static", f_na, kifmm.kifmm_evaluate_vjp_noalloc)):
        gc = torch.full((n,), float("nan"), device=dev)
        gp = torch.full((n, 3), float("nan"), device=dev)
        fn(f.plan, sd, wd, field, gc, gp, stream)
        torch.cuda.synchronize()
        out[label] = (gc.cpu().numpy(), gp.cpu().numpy())
    f_ref.close()
    f_na.close()
    return out


def test_no_alloc_derivative_matches_the_plan_workspace_form():
    # the per-parent leaf kernel and one stream for the upper levels on the no-allocation
    # plan, as on the reference plan's default choices where they differ in bits; the
    # U-list sum's workgroup size changes no bit
    for n, depth, p, seed, with_field in ((20_000, 3, 6, 5100, False), (3_000, 2, 4, 5200, True)):
        log(f"no-alloc vjp n={n} depth={depth} p={p} field={with_field}")
        out = _both(n, depth, p, seed, with_field)
        for k in (0, 1):
            a, b = out["plan"][k], out["static"][k]
            assert np.isfinite(b).all()
            rel = np.linalg.norm((a - b).astype(np.float64)) / np.linalg.norm(a.astype(np.float64))
            log(f"  output {k}: rel-L2 {rel:.3e}")
            assert rel < 1e-6


def test_no_alloc_derivative_rejects_large_plans():
    # one point over the limit (depth 5: about 64 points per leaf; one stream and forced
    # kernel forms, so that plan creation times nothing)
    import torch
    n = kifmm.KIFMM_NOALLOC_MAX_POINTS + 1
    log(f"no-alloc vjp size limit n={n}")
    x = workloads.points("cube", n, 5300)
    f = kifmm.FMM(x, 5, 3, cube=UNIT, flags=kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_SERIAL | kifmm.KIFMM_LEAF_BLOCKS |
                  kifmm.KIFMM_M2L_BLOCKED)
    dev = torch.device("cuda:0")
    s = torch.zeros(n, device=dev)
    gc = torch.zeros(n, device=dev)
    with pytest.raises(kifmm.KifmmError) as e:
        kifmm.kifmm_evaluate_vjp_noalloc(f.plan, s, s, None, gc, None)
    assert e.value.status == kifmm.KIFMM_E_INVALID and "at most" in str(e.value)
    f.close()
