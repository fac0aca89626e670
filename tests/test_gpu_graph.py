"""The evaluate captured in a HIP graph (through torch.cuda.graph) and replayed.

The evaluate issues only kernel launches and, with the side stream, event
record/wait pairs (no memset, no allocation, no host synchronisation), so a
captured evaluate must replay to the same bits as an eager one, including
after new charges are copied into the captured input buffer.  Each replay is
separated from the next by eager work and a synchronisation.
"""

import numpy as np
import pytest

from gpu_helpers import log
from paper_2604_19243_amd import kifmm, workloads

pytestmark = pytest.mark.gpu

UNIT = (0.5, 0.5, 0.5, 0.5)


@pytest.mark.parametrize("serial,nrhs,upper,queue", [(False, 1, False, False), (True, 1, False, False),
                                                     (False, 4, False, False), (False, 1, True, False),
                                                     (False, 1, False, True), (True, 1, False, True)])
def test_captured_evaluate_replays_bitwise(serial, nrhs, upper, queue):
    # upper: the levels above the leaves forced onto the plan's second stream (three streams captured);
    # queue: the persistent leaf kernel, whose work-queue counters a kernel clears in every replay
    import torch
    log(f"graph capture serial={serial} nrhs={nrhs} upper={upper} queue={queue}")
    n, depth, p = 20_000, 4 if upper else 3, 6
    x = workloads.points("cube", n, 1001)
    flags = kifmm.KIFMM_POTENTIAL | (kifmm.KIFMM_SERIAL if serial else 0)
    flags |= kifmm.KIFMM_GRADIENT if nrhs == 1 else 0
    flags |= kifmm.KIFMM_UPPER_STREAM if upper else 0
    flags |= kifmm.KIFMM_LEAF_QUEUE if queue else (kifmm.KIFMM_LEAF_BLOCKS if nrhs == 1 else 0)
    f = kifmm.FMM(x, depth, p, cube=UNIT, flags=flags, nrhs=nrhs)
    dev = torch.device("cuda:0")
    shape = (n,) if nrhs == 1 else (n, nrhs)
    rng = np.random.default_rng(5)
    charge_sets = [torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).to(dev) for _ in range(3)]
    q = charge_sets[0].clone()
    pot = torch.zeros(shape, device=dev)
    grad = torch.zeros(n, 3, device=dev) if nrhs == 1 else None
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        f.evaluate(q, pot, grad, stream=s.cuda_stream)   # warm-up (kernel attributes set eagerly)
    torch.cuda.synchronize()
    if upper:
        assert kifmm.kifmm_plan_get_stats(f.plan)["upper_stream"] == 1
    assert kifmm.kifmm_plan_get_stats(f.plan)["leaf_queue"] == (1 if queue else 0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        f.evaluate(q, pot, grad, stream=s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        q.copy_(charge_sets[rep])
        pot.zero_()
        if grad is not None:
            grad.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_p = pot.clone()
        got_g = grad.clone() if grad is not None else None
        # eager evaluate of the same charges, into fresh buffers
        ep = torch.zeros(shape, device=dev)
        eg = torch.zeros(n, 3, device=dev) if grad is not None else None
        f.evaluate(charge_sets[rep], ep, eg)
        torch.cuda.synchronize()
        assert torch.equal(got_p, ep), f"replay {rep}: potentials differ from eager"
        if grad is not None:
            assert torch.equal(got_g, eg), f"replay {rep}: gradients differ from eager"
    del g
    f.close()
