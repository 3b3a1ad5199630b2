"""Pins of the NumPy PPPM-ik oracle.

The mesh method has no printed worked example in the paper either.  Its parts
are pinned by textbook values of the cardinal B-splines (Eulerian numbers),
by the moment identities of B-spline assignment, by properties of the optimal
influence function, by exact symmetries of the discrete method (integer mesh
shifts, zero net force) and, end to end, by convergence to the direct Ewald
oracle at the rate the assignment order predicts.
"""
import math

import numpy as np
import pytest

import systems
from oracle import pppm

KE = systems.COULOMB_K
BETA = systems.BETA


@pytest.fixture(scope="module")
def w64():
    return systems.workload(1).system()


@pytest.fixture(scope="module")
def ewald64(ewald, w64):
    e, w, fi, fw = ewald.system_recip(w64, BETA, KE)
    return e, w, np.concatenate([fi, fw])


# M_p at the integers 1..p-1 are the Eulerian numbers A(p-1, k) / (p-1)!.
EULERIAN = {
    2: [1],
    3: [1, 1],
    4: [1, 4, 1],
    5: [1, 11, 11, 1],
    6: [1, 26, 66, 26, 1],
    7: [1, 57, 302, 302, 57, 1],
    8: [1, 120, 1191, 2416, 1191, 120, 1],
}


@pytest.mark.parametrize("p", sorted(EULERIAN))
def test_bspline_integer_values(p):
    x = np.arange(1, p)
    expect = np.array(EULERIAN[p], float) / math.factorial(p - 1)
    assert np.allclose(pppm.bspline(p, x), expect, rtol=0, atol=1e-15)
    assert pppm.bspline(p, 0.0) == 0.0 and pppm.bspline(p, float(p)) == 0.0


def test_quartic_bspline_half_integers():
    # centred quartic B-spline at 0, +-1, +-2: 115/192, 19/96, 1/384
    v = pppm.bspline(5, np.array([2.5, 1.5, 3.5, 0.5, 4.5]))
    assert np.allclose(v, [115 / 192, 19 / 96, 19 / 96, 1 / 384, 1 / 384], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8])
def test_assignment_moments(p):
    """Sum of weights = 1, first moment reproduces u, second central moment = p/12."""
    rng = np.random.default_rng(p)
    u = rng.uniform(10, 20, 1000)
    g, w = pppm.stencil(u, p)
    assert np.allclose(w.sum(1), 1.0, atol=1e-14)
    assert np.allclose((g * w).sum(1), u, atol=1e-12)
    assert np.allclose(((g - u[:, None]) ** 2 * w).sum(1), p / 12.0, atol=1e-12)
    assert (w >= 0).all()
    assert (np.abs(g - u[:, None]) <= p / 2).all()


def test_spread_conserves_charge_and_dipole():
    rng = np.random.default_rng(3)
    box = np.array([10.0, 12.0, 14.0])
    K = (16, 16, 32)
    pos = rng.uniform(3, 7, (20, 3))          # away from the periodic seam
    q = rng.normal(size=20)
    Q = pppm.spread(pos, q, box, K, 5)
    assert abs(Q.sum() - q.sum()) < 1e-12
    h = box / np.array(K)
    for a in range(3):
        g = np.arange(K[a]).reshape([-1 if i == a else 1 for i in range(3)])
        assert abs((Q * g).sum() - (q * pos[:, a] / h[a]).sum()) < 1e-11


def test_influence_symmetry_and_continuum_limit():
    box = np.array([20.0, 20.0, 20.0])
    K = (64, 64, 64)
    G = pppm.influence(box, K, BETA, 5)
    assert G[0, 0, 0] == 0.0
    # even in every component separately
    # n -> -n on one axis is index i -> (K - i) mod K
    assert np.allclose(G, np.roll(G[::-1], 1, 0), rtol=1e-13, atol=0)
    assert np.allclose(G, np.roll(G[:, ::-1], 1, 1), rtol=1e-13, atol=0)
    assert np.allclose(G, np.roll(G[:, :, ::-1], 1, 2), rtol=1e-13, atol=0)
    # axis permutation symmetry of a cubic box
    assert np.allclose(G, G.transpose(1, 0, 2), rtol=1e-13, atol=0)
    # small k h: G -> phi(k) / U(k)^2
    k = 2 * math.pi / 20.0
    h = 20.0 / 64
    phi = 4 * math.pi * math.exp(-k * k / (4 * BETA * BETA)) / (k * k)
    U = (math.sin(k * h / 2) / (k * h / 2)) ** 5
    assert abs(G[1, 0, 0] - phi / U ** 2) / G[1, 0, 0] < 1e-6


def test_influence_alias_range_converged():
    box = np.array([32.325] * 3)
    g2 = pppm.influence(box, (32, 32, 32), BETA, 5, alias=2)
    g3 = pppm.influence(box, (32, 32, 32), BETA, 5, alias=3)
    assert np.abs(g3 - g2).max() / np.abs(g2).max() < 1e-10


def test_converges_to_ewald_at_order_p(w64, ewald64):
    e0, w0, f0 = ewald64
    errs = []
    for K in (16, 32, 64):
        E, F, W = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, (K,) * 3, 5, BETA, KE)
        errs.append(pppm.rel_rmse(F, f0))
    # halving h cuts the force error by ~2^p (p = 5); require at least 2^4
    assert errs[0] / errs[1] > 16 and errs[1] / errs[2] > 16


def test_refined_mesh_matches_ewald_to_1e9(w64, ewald64):
    e0, w0, f0 = ewald64
    E, F, W = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, (64,) * 3, 8, BETA, KE)
    assert abs(E - e0) / abs(e0) < 1e-9
    assert pppm.rel_rmse(F, f0) < 1e-9
    assert np.abs(W - w0).max() / abs(e0) < 1e-9


def test_integer_mesh_shift_is_exact(w64):
    K = (32, 32, 32)
    h = w64.box / 32
    pos, q = w64.all_pos(), w64.all_q()
    E, F, W = pppm.pppm(pos, q, w64.box, K, 5, BETA, KE)
    shift = h * np.array([3, -7, 11])
    E2, F2, W2 = pppm.pppm(np.mod(pos + shift, w64.box), q, w64.box, K, 5, BETA, KE)
    assert abs(E2 - E) / abs(E) < 1e-13
    assert np.abs(F2 - F).max() / np.abs(F).max() < 1e-12
    assert np.abs(W2 - W).max() / abs(E) < 1e-13


def test_zero_net_force(w64):
    E, F, W = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, (32,) * 3, 5, BETA, KE)
    assert np.linalg.norm(F.sum(0)) / np.abs(F).max() < 1e-12


def test_real_fields(w64):
    """With the Nyquist derivative removed the three fields are real."""
    _, _, _, parts = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, (16, 16, 16), 5, BETA, KE,
                               return_parts=True)
    for a in range(3):
        kd = np.fft.fftfreq(16, 1 / 16)
        kd = np.where(kd == -8, 0.0, 2 * math.pi * kd / w64.box[a])
        shape = [1, 1, 1]
        shape[a] = 16
        Eh = -1j * kd.reshape(shape) * parts["G"] * parts["Qhat"]
        Ea = np.fft.ifftn(Eh) * 16 ** 3
        assert np.abs(Ea.imag).max() < 1e-12 * np.abs(Ea.real).max()


# ---------------------------------------------------------------------------
# Analytic-differentiation variant: its forces are the exact gradient of the
# PPPM energy, so central finite differences of pppm()'s energy pin every
# step of it (spread, transforms, influence function, derivative weights,
# normalisation and sign).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_bspline_derivative_matches_finite_differences(p):
    x = np.linspace(0.013, p - 0.017, 97)
    h = 1e-6
    fd = (pppm.bspline(p, x + h) - pppm.bspline(p, x - h)) / (2 * h)
    assert np.abs(pppm.dbspline(p, x) - fd).max() < 1e-8


@pytest.mark.parametrize("p", [3, 5, 8])
def test_ad_forces_are_the_energy_gradient(p):
    s = systems.workload(1).system()
    pos, q, box = s.all_pos(), s.all_q(), s.box
    K = (16, 16, 16)
    G = pppm.influence(box, K, BETA, p)
    E, F, W = pppm.pppm_ad(pos, q, box, K, p, BETA, KE, G=G)
    E_ik = pppm.pppm(pos, q, box, K, p, BETA, KE, G=G)[0]
    assert abs(E - E_ik) <= 1e-14 * abs(E)
    step = 1e-5
    for j in (0, 7, 100, s.n - 1):
        for a in range(3):
            d = []
            for sg in (1, -1):
                r = pos.copy()
                r[j, a] += sg * step
                d.append(pppm.pppm_ad(r, q, box, K, p, BETA, KE, G=G)[0])
            fd = -(d[0] - d[1]) / (2 * step)
            # measured ~1e-9 (FD truncation and rounding); the ik forces of the
            # same energy differ by 3e-4 (p = 5) to 6e-6 (p = 8)
            assert abs(F[j, a] - fd) <= 1e-8 * np.abs(F[j]).max()


# ---------------------------------------------------------------------------
# Meshes that are not powers of two (the paper's precision study uses grids
# such as 10x15x10): odd sizes have no Nyquist index, even ones drop its
# derivative.  The exact symmetries and the convergence to Ewald must hold
# for them as for the power-of-two meshes.
# ---------------------------------------------------------------------------
MIXED = (15, 18, 25)


def test_mixed_mesh_integer_shift_and_zero_net_force(w64):
    pos, q = w64.all_pos(), w64.all_q()
    E, F, W = pppm.pppm(pos, q, w64.box, MIXED, 5, BETA, KE)
    assert np.linalg.norm(F.sum(0)) / np.abs(F).max() < 1e-12
    shift = (w64.box / np.array(MIXED)) * np.array([4, -5, 13])
    E2, F2, W2 = pppm.pppm(np.mod(pos + shift, w64.box), q, w64.box, MIXED, 5, BETA, KE)
    assert abs(E2 - E) / abs(E) < 1e-13
    assert np.abs(F2 - F).max() / np.abs(F).max() < 1e-12
    assert np.abs(W2 - W).max() / abs(E) < 1e-13


def test_mixed_mesh_fields_are_real(w64):
    _, _, _, parts = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, MIXED, 5, BETA, KE, return_parts=True)
    for a in range(3):
        n = np.fft.fftfreq(MIXED[a], 1 / MIXED[a])
        kd = 2 * math.pi * n / w64.box[a]
        if MIXED[a] % 2 == 0:
            kd = np.where(n == -MIXED[a] // 2, 0.0, kd)
        shape = [1, 1, 1]
        shape[a] = MIXED[a]
        Ea = np.fft.ifftn(-1j * kd.reshape(shape) * parts["G"] * parts["Qhat"])
        assert np.abs(Ea.imag).max() < 1e-12 * np.abs(Ea.real).max()


def test_mixed_meshes_converge_to_ewald(w64, ewald64):
    e0, w0, f0 = ewald64
    errs = []
    for K in ((15, 15, 15), (30, 30, 30), (60, 60, 60)):
        E, F, W = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, K, 5, BETA, KE)
        errs.append(pppm.rel_rmse(F, f0))
    assert errs[0] / errs[1] > 16 and errs[1] / errs[2] > 16
    E, F, W = pppm.pppm(w64.all_pos(), w64.all_q(), w64.box, (75, 75, 75), 8, BETA, KE)
    assert abs(E - e0) / abs(e0) < 1e-9
    assert pppm.rel_rmse(F, f0) < 1e-9
