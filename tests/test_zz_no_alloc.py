"""The step without device allocation (dplr_lr_compute_noalloc) against the
plan entry point (dplr_lr_compute_energy_forces_virial) on the same inputs.

Both run the same kernels on the same launch shapes, so the results are
expected to agree bitwise; the assertion uses the parity bars of the plan
path (FP64: 1e-10 relative force RMSE, FP32: 1e-5; energy and virial 1e-12
and 2e-6) so that a legitimate difference in summation order would still be
judged by the same standard as every other parity test.  Each test makes two
calls in a row, the second with fewer particles, so that stale contents of
the shared scratch array from the first call cannot go unnoticed.  The last
two checks are host-side rejections (no device work)."""
import numpy as np
import pytest

import systems

pytestmark = pytest.mark.gpu

KE = systems.COULOMB_K
BETA = systems.BETA


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.fixture(scope="module")
def dl():
    import paper_2504_15508_amd as m
    return m


def _rel(a, b):
    a = a.double().cpu().numpy().ravel()
    b = b.double().cpu().numpy().ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _compare(torch, dl, s, mesh, order, precision, n_keep, diff="ik"):
    """Plan path and no-allocation path on the first n_keep ions and WCs."""
    dt = torch.float64 if precision == "fp64" else torch.float32
    ni, nw = n_keep
    ip = torch.tensor(s.ion_pos[:ni], dtype=dt, device="cuda").contiguous()
    iq = torch.tensor(s.ion_q[:ni], dtype=dt, device="cuda").contiguous()
    wp = torch.tensor(s.wc_pos[:nw], dtype=dt, device="cuda").contiguous()
    wq = torch.tensor(s.wc_q[:nw], dtype=dt, device="cuda").contiguous()
    # the no-allocation call first: it must raise the kernels' LDS limits itself
    E1, fi1, fw1, W1 = dl.plan.compute_noalloc(mesh, s.box, ip, iq, wp, wq, order=order, beta=BETA,
                                               coulomb_k=KE, diff=diff)
    plan = dl.Plan(mesh, order=order, beta=BETA, coulomb_k=KE, precision=precision, capacity=ni + nw, diff=diff)
    plan.set_box(s.box)
    E0, fi0, fw0, W0 = plan.compute(ip, iq, wp, wq)
    torch.cuda.synchronize()
    plan.close()
    bitwise = bool(torch.equal(fi0, fi1) and torch.equal(fw0, fw1) and torch.equal(E0, E1) and torch.equal(W0, W1))
    F0 = torch.cat([fi0, fw0])
    F1 = torch.cat([fi1, fw1])
    dF = _rel(F1, F0)
    dE = abs(float(E1) - float(E0)) / abs(float(E0))
    dW = float((W1 - W0).abs().max()) / abs(float(E0))
    print(f"noalloc {precision} mesh {mesh} order {order} {diff} n={ni + nw}: dF={dF:.1e} dE={dE:.1e} "
          f"dW={dW:.1e} bitwise={bitwise}", flush=True)
    fbar, ebar = (1e-10, 1e-12) if precision == "fp64" else (1e-5, 2e-6)
    assert dF <= fbar and dE <= ebar and dW <= ebar
    assert torch.isfinite(F1).all()


@pytest.mark.parametrize("precision,mesh", [("fp32", 64), ("fp64", 32)])
def test_noalloc_matches_plan_two_calls(torch, dl, precision, mesh):
    wl = systems.workload(2 if mesh == 64 else 1)
    s = wl.system()
    ni, nw = len(s.ion_q), len(s.wc_q)
    _compare(torch, dl, s, mesh, 5, precision, (ni, nw))
    # second call: fewer particles (the scratch array keeps the first call's contents)
    _compare(torch, dl, s, mesh, 5, precision, (ni // 2, nw // 3))


def test_noalloc_mesh_and_order_change(torch, dl):
    """A different mesh, order and force scheme after the calls above (new
    influence table and layout), then the benchmark system at 128^3."""
    s = systems.workload(2).system()
    _compare(torch, dl, s, 32, 7, "fp32", (len(s.ion_q), len(s.wc_q)), diff="ad")
    s3 = systems.workload(3).system()
    _compare(torch, dl, s3, 128, 5, "fp32", (len(s3.ion_q), len(s3.wc_q)))
    _compare(torch, dl, s3, 128, 5, "fp32", (len(s3.ion_q) // 4, len(s3.wc_q) // 4))


def test_noalloc_rejects_oversize_and_mixed(torch, dl):
    s = systems.workload(1).system()
    ip = torch.tensor(s.ion_pos, dtype=torch.float32, device="cuda")
    iq = torch.tensor(s.ion_q, dtype=torch.float32, device="cuda")
    with pytest.raises(dl.DplrError) as ei:
        dl.plan.compute_noalloc(256, s.box, ip, iq)
    assert ei.value.status == dl._lib.E_CAPACITY and "scratch" in str(ei.value)
    with pytest.raises(dl.DplrError) as ei:
        dl.plan.compute_noalloc((12, 18, 12), s.box, ip, iq)
    assert ei.value.status == dl._lib.E_UNSUPPORTED
