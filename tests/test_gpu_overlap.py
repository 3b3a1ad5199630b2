"""The long-range step on its own stream beside other GPU work.

The step is launched on a side stream while a stand-in short-range workload
(bf16 GEMMs) runs on another stream at the same time, as a caller overlapping
the long-range and short-range parts of a DPLR step would do.  Its results
must equal those of the step run alone, bitwise (FP32 mesh sums are fixed
point, so sharing the GPU cannot change them).
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


def test_step_beside_other_streams_matches_isolated(torch_dev):
    torch = torch_dev
    import paper_2504_15508_amd as dl
    s = systems.workload(2).system()
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ri, qi, rw, qw = t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q)
    s_lr, s_sr = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s_lr):
        plan = dl.Plan(64, order=5, precision="fp32", capacity=s.n)
        plan.set_box(s.box)
        ref = [x.clone() for x in plan.compute(ri, qi, rw, qw)]
    torch.cuda.synchronize()
    a = torch.randn(4096, 1024, device="cuda").bfloat16()
    b = torch.randn(1024, 1024, device="cuda").bfloat16()
    for _ in range(3):
        with torch.cuda.stream(s_sr):
            for _ in range(8):
                c = a @ b
        with torch.cuda.stream(s_lr):
            out = plan.compute(ri, qi, rw, qw)
        torch.cuda.synchronize()
        for x, y in zip(out, ref):
            assert torch.equal(x, y)
        assert torch.isfinite(c.float()).all()
    plan.close()
