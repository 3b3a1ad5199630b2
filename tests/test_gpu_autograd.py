"""The torch.autograd.Function: its backward returns dE/dr of ions and WCs
computed by the library.  Checked against central finite differences of the
oracle energy, against the oracle's analytic gradient, and through a
synthetic differentiable WC model W_n(R) (the chain the Deep Wannier model
takes back to the atoms)."""
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


def test_backward_is_minus_g_times_force(torch):
    import paper_2504_15508_amd as dl
    s = systems.workload(1).system()
    p = dl.Plan(32, order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    p.set_box(s.box)
    t = lambda a, g=False: torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=g)
    ri, rw = t(s.ion_pos, True), t(s.wc_pos, True)
    E = dl.dplr_long_range(ri, rw, t(s.ion_q), t(s.wc_q), p)
    (2.5 * E).backward()
    _, fi, fw, _ = p.compute(t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q))
    assert torch.allclose(ri.grad, -2.5 * fi, rtol=1e-12, atol=1e-12)
    assert torch.allclose(rw.grad, -2.5 * fw, rtol=1e-12, atol=1e-12)


def test_config2_gradient_vs_oracle_fd_and_analytic(torch):
    """FP32 backward at config 2 (64^3, order 5) on 32 seeded particles versus
    central finite differences (h = 1e-4 A, FP64) of the Ewald energy and the
    oracle's analytic forces (stored by tests/golden/make_golden.py fd).  ik
    forces equal the exact gradient only up to the mesh's discretisation
    error, so the bar is the measured method error of this mesh (3.9e-4
    relative RMSE over all forces) with margin."""
    import json
    import os
    import paper_2504_15508_amd as dl
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ewald_fd_water4096_fp32.json")))
    s = systems.workload(2).system().rounded(np.float32)
    p = dl.Plan(64, order=5, beta=BETA, coulomb_k=KE, precision="fp32", capacity=s.n)
    p.set_box(s.box)
    t = lambda a, g=False: torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=g)
    ri, rw = t(s.ion_pos, True), t(s.wc_pos, True)
    E = dl.dplr_long_range(ri, rw, t(s.ion_q), t(s.wc_q), p)
    E.backward()
    grad = np.concatenate([ri.grad.double().cpu().numpy(), rw.grad.double().cpu().numpy()])
    idx = np.array(gold["index"])
    fd, f_or = np.array(gold["fd_gradient"]), np.array(gold["oracle_force"])
    g = grad[idx]
    rel_fd = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    rel_an = np.linalg.norm(g + f_or) / np.linalg.norm(f_or)
    fd_vs_an = np.linalg.norm(fd + f_or) / np.linalg.norm(f_or)
    print(f"grad vs FD {rel_fd:.2e}, vs oracle gradient {rel_an:.2e}, FD vs oracle {fd_vs_an:.2e}")
    assert fd_vs_an < 1e-7
    assert rel_fd < 1.5e-3 and rel_an < 1.5e-3


def test_chain_through_synthetic_wannier_model(torch):
    """W_n = R_O(n) + Delta_n(R) with a smooth synthetic Delta; autograd chains
    the WC gradient into the atoms.  Compared with finite differences of the
    energy evaluated through the same GPU path in FP64 at a fine mesh."""
    import paper_2504_15508_amd as dl
    s = systems.workload(1).system()
    p = dl.Plan(64, order=8, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    p.set_box(s.box)
    ion0 = torch.tensor(s.ion_pos, dtype=torch.float64, device="cuda")
    qi = torch.tensor(s.ion_q, dtype=torch.float64, device="cuda")
    qw = torch.tensor(s.wc_q, dtype=torch.float64, device="cuda")

    def energy(ion):
        o, h1, h2 = ion[0::3], ion[1::3], ion[2::3]
        bis = (h1 + h2) * 0.5 - o
        delta = 0.25 * bis / bis.norm(dim=1, keepdim=True) * (1 + 0.1 * torch.tanh(o[:, :1] - 6.0))
        return dl.dplr_long_range(ion, o + delta, qi, qw, p)

    ion = ion0.clone().requires_grad_(True)
    energy(ion).backward()
    g = ion.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    h = 1e-5
    errs = []
    for j in rng.choice(s.n_ion, 6, replace=False):
        for a in range(3):
            e = []
            for sg in (1, -1):
                x = ion0.clone()
                x[j, a] += sg * h
                e.append(float(energy(x)))
            fd = (e[0] - e[1]) / (2 * h)
            errs.append(abs(fd - g[j, a]) / max(1.0, abs(g).max()))
    print(f"chain rule max err {max(errs):.2e}")
    assert max(errs) < 1e-6


def test_chain_through_synthetic_wannier_model_vs_oracle(torch):
    """The same chain against the oracle: the expected atom gradient is
    -F_ion - J^T F_wc, with F_ion, F_wc the FP64 PPPM oracle's forces at the
    atoms and at the WCs W(R), and J = dW/dR the Jacobian of the synthetic
    Delta (its vector-Jacobian product taken by torch on the CPU; no GPU
    value enters the expectation).  Same mesh and order on both sides, so the
    bar is the FP64 parity bar."""
    import paper_2504_15508_amd as dl
    from oracle import pppm
    s = systems.workload(1).system()
    mesh, order = 32, 6
    p = dl.Plan(mesh, order=order, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    p.set_box(s.box)

    def wannier(ion):
        o, h1, h2 = ion[0::3], ion[1::3], ion[2::3]
        bis = (h1 + h2) * 0.5 - o
        return o + 0.25 * bis / bis.norm(dim=1, keepdim=True) * (1 + 0.1 * torch.tanh(o[:, :1] - 6.0))

    qi = torch.tensor(s.ion_q, dtype=torch.float64, device="cuda")
    qw = torch.tensor(s.wc_q, dtype=torch.float64, device="cuda")
    ion = torch.tensor(s.ion_pos, dtype=torch.float64, device="cuda", requires_grad=True)
    dl.dplr_long_range(ion, wannier(ion), qi, qw, p).backward()
    g = ion.grad.cpu().numpy()

    ion_c = torch.tensor(s.ion_pos, dtype=torch.float64, requires_grad=True)   # CPU
    w_c = wannier(ion_c)
    pos = np.concatenate([s.ion_pos, w_c.detach().numpy()])
    q = np.concatenate([s.ion_q, s.wc_q])
    _, F0, _ = pppm.pppm(pos, q, s.box, (mesh,) * 3, order, BETA, KE)
    F_ion, F_wc = F0[: s.n_ion], F0[s.n_ion:]
    (jt,) = torch.autograd.grad(w_c, ion_c, grad_outputs=torch.tensor(-F_wc, dtype=torch.float64))
    expect = -F_ion + jt.numpy()
    err = float(np.linalg.norm(g - expect) / np.linalg.norm(expect))
    err_max = float(np.abs(g - expect).max() / np.abs(expect).max())
    # the WC term must matter: dropping it changes the gradient at O(1)
    drop = float(np.linalg.norm(-F_ion - expect) / np.linalg.norm(expect))
    print(f"chain rule vs oracle: rel {err:.2e}, max {err_max:.2e} (without the WC term: {drop:.2e})")
    assert err <= 1e-9 and err_max <= 1e-9
    assert drop > 1e-2
