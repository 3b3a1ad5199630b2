"""GPU parity of the analytic-differentiation (ad) variant against the oracle.

The ad plans share the sort, spread, forward transforms, influence function,
energy and virial with the ik plans; the z pass then forms the potential
spectrum G Q^ alone, one inverse plane pass gives the potential, and the
gather applies the derivatives of the B-spline weights.  Its forces are the
exact gradient of the PPPM energy, so besides the oracle comparison they must
match finite differences of the plan's own FP64 energy (which the ik forces
of the same energy do not, by the method's discretisation error).
"""
import numpy as np
import pytest

import systems
from oracle import pppm

pytestmark = pytest.mark.gpu

KE = systems.COULOMB_K
BETA = systems.BETA
FP32_TOL_F, FP32_TOL_E = 1e-5, 2e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


def run(torch, sys, mesh, order, precision, diff="ad", flags=0):
    import paper_2504_15508_amd as dl
    dt = torch.float64 if precision == "fp64" else torch.float32
    mesh = (mesh,) * 3 if isinstance(mesh, int) else tuple(mesh)
    plan = dl.Plan(mesh, order=order, beta=BETA, coulomb_k=KE, precision=precision,
                   capacity=sys.n, flags=flags, diff=diff)
    plan.set_box(sys.box)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    E, fi, fw, W = plan.compute(t(sys.ion_pos), t(sys.ion_q), t(sys.wc_pos), t(sys.wc_q))
    torch.cuda.synchronize()
    out = (float(E.item()), np.concatenate([fi.double().cpu().numpy(), fw.double().cpu().numpy()]),
           W.cpu().numpy())
    plan.close()
    return out


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def check(torch, sys, mesh, order, precision, tol_f, tol_e):
    E, F, W = run(torch, sys, mesh, order, precision)
    ref = sys.rounded(np.float32) if precision == "fp32" else sys
    K = (mesh,) * 3 if isinstance(mesh, int) else tuple(mesh)
    E0, F0, W0 = pppm.pppm_ad(ref.all_pos(), ref.all_q(), ref.box, K, order, BETA, KE)
    dE, dF, dW = abs(E - E0) / abs(E0), rel(F, F0), np.abs(W - W0).max() / abs(E0)
    print(f"ad {sys.name} K={mesh} p={order} {precision}: dE={dE:.2e} dF={dF:.2e} dW={dW:.2e}", flush=True)
    assert dE <= tol_e
    assert dF <= tol_f
    assert dW <= tol_e


@pytest.mark.parametrize("order", [2, 3, 5, 8])
def test_ad_fp64_matches_oracle(torch_dev, order):
    check(torch_dev, systems.workload(1).system(), 32, order, "fp64", 1e-10, 1e-10)


def test_ad_fp32_config2_matches_oracle(torch_dev):
    check(torch_dev, systems.workload(2).system(), 64, 5, "fp32", FP32_TOL_F, FP32_TOL_E)


def test_ad_full_size_fp32_matches_oracle(torch_dev):
    # the 216k system at 128^3, in the configuration the benchmark's ad leg times
    check(torch_dev, systems.workload(3).system(), 128, 5, "fp32", FP32_TOL_F, FP32_TOL_E)


@pytest.mark.parametrize("mesh", [(256, 64, 32), (16, 128, 64)])
def test_ad_fp32_noncubic_matches_oracle(torch_dev, mesh):
    s = systems.water_box(100, 14.0, seed=99)
    s.box = np.array([14.0, 18.0, 11.0])
    s.ion_pos = np.mod(s.ion_pos, s.box)
    s.wc_pos = np.mod(s.wc_pos, s.box)
    check(torch_dev, s, mesh, 5, "fp32", FP32_TOL_F, FP32_TOL_E)


def test_ad_energy_and_virial_equal_ik(torch_dev):
    """Same spread, transforms and reductions: bitwise the same energy and virial."""
    s = systems.workload(2).system()
    Ea, _, Wa = run(torch_dev, s, 64, 5, "fp32", diff="ad")
    Ei, _, Wi = run(torch_dev, s, 64, 5, "fp32", diff="ik")
    assert Ea == Ei
    assert np.array_equal(Wa, Wi)


def test_ad_forces_are_the_gradient_of_the_plan_energy(torch_dev):
    """Central differences (h = 2e-4 A) of the FP64 plan's own energy on a
    16^3 mesh against its ad forces; the ik forces of the same energy miss
    this bar by orders of magnitude (their difference is the method's
    discretisation error, ~3e-4 here).  The bar covers the FD truncation
    error (h^2/6 times the third derivative of the piecewise-cubic force,
    ~1e-7 of F at a 0.78 A spacing) and the energy's rounding (the 2^-40
    fixed-point mesh, ~1e-12 of E, divided by 2h)."""
    import copy
    s = systems.workload(1).system()
    _, F, _ = run(torch_dev, s, 16, 5, "fp64")
    _, Fik, _ = run(torch_dev, s, 16, 5, "fp64", diff="ik")
    step = 2e-4
    worst, worst_ik = 0.0, 0.0
    for j in (0, 5, 77, s.n - 1):
        for a in range(3):
            e = []
            for sg in (1, -1):
                t = copy.deepcopy(s)
                if j < s.n_ion:
                    t.ion_pos[j, a] += sg * step
                else:
                    t.wc_pos[j - s.n_ion, a] += sg * step
                e.append(run(torch_dev, t, 16, 5, "fp64")[0])
            fd = -(e[0] - e[1]) / (2 * step)
            scale = np.abs(F[j]).max()
            worst = max(worst, abs(F[j, a] - fd) / scale)
            worst_ik = max(worst_ik, abs(Fik[j, a] - fd) / scale)
    print(f"ad vs FD of the plan energy: {worst:.2e} (ik: {worst_ik:.2e})", flush=True)
    assert worst <= 2e-6
    assert worst_ik > 1e-4


def test_ad_longest_rows_match_oracle(torch_dev):
    # 512-point x rows: the LDS Stockham transforms and unfused passes
    s = systems.water_box(100, 14.0, seed=99)
    s.box = np.array([24.0, 12.0, 12.0])
    s.ion_pos = np.mod(s.ion_pos, s.box)
    s.wc_pos = np.mod(s.wc_pos, s.box)
    check(torch_dev, s, (512, 16, 32), 5, "fp32", FP32_TOL_F, FP32_TOL_E)


# meshes whose z planes do not fit in LDS: pencil spread, separate inverse y
# and x passes writing the padded potential
@pytest.mark.parametrize("precision,tol_f,tol_e", [("fp64", 1e-10, 1e-10), ("fp32", FP32_TOL_F, FP32_TOL_E)])
def test_ad_pencil_path_matches_oracle(torch_dev, precision, tol_f, tol_e):
    check(torch_dev, systems.workload(1).system(), (256, 128, 16), 5, precision, tol_f, tol_e)
