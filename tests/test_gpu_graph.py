"""The long-range step under HIP graph capture (as the benchmark times it).

One call of the step is captured in a graph and replayed several times, with
unrelated eager GPU work and host synchronisation between the replays; every
replay must reproduce the eager call bitwise (the FP32 mesh is accumulated in
fixed point, so the step is deterministic).  The step enqueues no memset or
copy, only kernels, so nothing in it depends on replay-time state.
"""
import numpy as np
import pytest

import systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_graph_replays_match_eager(torch_dev, diff):
    torch = torch_dev
    import paper_2504_15508_amd as dl
    s = systems.workload(2).system()
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ri, qi, rw, qw = t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = dl.Plan(64, order=5, precision="fp32", capacity=s.n, diff=diff)
        plan.set_box(s.box)
        ref = [x.clone() for x in plan.compute(ri, qi, rw, qw)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        out = plan.compute(ri, qi, rw, qw)
    for r in range(3):
        a = torch.randn(512, 512, device="cuda")
        (a @ a).sum().item()              # unrelated eager work and a host sync
        for x in out:
            x.zero_()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out, ref):
            assert torch.equal(x, y), f"replay {r} differs from the eager call"
    plan.close()


@pytest.mark.parametrize("int32", [False, True])
def test_graph_replays_match_eager_mixed_radix(torch_dev, int32):
    # the mixed-radix kernels clear their fixed-point mesh themselves (no
    # memset), so captured replays start from a clean mesh too
    torch = torch_dev
    import paper_2504_15508_amd as dl
    s = systems.water_box(128, 16.0, seed=20261128)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ri, qi, rw, qw = t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = dl.Plan((12, 18, 12), order=5, precision="fp32", capacity=s.n)
        plan.set_box(s.box)
        if int32:
            plan.set_fft_int32((2, 3, 2), 1e7)
        ref = [x.clone() for x in plan.compute(ri, qi, rw, qw)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        out = plan.compute(ri, qi, rw, qw)
    for r in range(3):
        a = torch.randn(512, 512, device="cuda")
        (a @ a).sum().item()
        for x in out:
            x.zero_()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out, ref):
            assert torch.equal(x, y), f"replay {r} differs from the eager call"
    plan.close()
