"""Pins of the FP64 Ewald oracle against mathematics it must reproduce.

The paper prints no worked example of the long-range energy, so the oracle is
pinned by closed forms (the NaCl Madelung constant, the isolated-pair limit),
by exact invariances (zero net force, translation), by its own derivatives
(finite differences of the energy for forces and, under strain, for the
virial), by cutoff convergence and by an independent NumPy twin.
"""
import math

import numpy as np
import pytest

import systems
from oracle import ewald_np

KE = systems.COULOMB_K
BETA = systems.BETA
# NaCl (rock salt) Madelung constant referred to the nearest-neighbour distance;
# the literature value to 14 digits and the 7-digit figure 1.747565.
MADELUNG_NACL = 1.74756459463318


@pytest.fixture(scope="module")
def w64():
    return systems.workload(1).system()


def _madelung(ew, beta):
    c = systems.nacl_crystal(2, a=5.64)
    e = ew.full_energy(c.all_pos(), c.all_q(), c.box, beta, KE)
    n_pairs = c.n // 2
    r0 = 5.64 / 2
    return -e * r0 / (n_pairs * KE)


def test_madelung_nacl(ewald):
    m = _madelung(ewald, 0.4)
    assert abs(m - MADELUNG_NACL) / MADELUNG_NACL < 1e-10
    assert abs(m - 1.747565) < 1e-6


@pytest.mark.parametrize("beta", [0.2, 0.3, 0.5])
def test_full_ewald_independent_of_beta(ewald, beta):
    c = systems.nacl_crystal(2, a=5.64)
    e0 = ewald.full_energy(c.all_pos(), c.all_q(), c.box, 0.4, KE)
    e1 = ewald.full_energy(c.all_pos(), c.all_q(), c.box, beta, KE)
    assert abs(e1 - e0) / abs(e0) < 1e-10


def test_isolated_pair_limit(ewald):
    """A +q/-q pair at separation r in a box L >> r: the Gaussian-charge energy
    tends to k_e q^2 (2 beta/sqrt(pi) - erf(beta r)/r); the image dipoles leave
    a residual of order r^2/L^3."""
    r = 1.0
    res = []
    for L in (20.0, 40.0):
        pos = np.array([[L / 2, L / 2, L / 2], [L / 2 + r, L / 2, L / 2]])
        q = np.array([1.0, -1.0])
        e, _, _ = ewald.recip(pos, q, [L, L, L], BETA, KE, forces=False)
        limit = KE * (2 * BETA / math.sqrt(math.pi) - math.erf(BETA * r) / r)
        res.append(e - limit)
    assert abs(res[1]) < 2e-4 * KE
    # residual falls as 1/L^3 (within 10 %)
    assert 7.2 < res[0] / res[1] < 8.8


def test_twin_agrees(ewald, w64):
    e, w, fi, fw = ewald.system_recip(w64, BETA, KE)
    e2, w2, f2 = ewald_np.recip(w64.all_pos(), w64.all_q(), w64.box, BETA, KE, ewald.mcut_for(BETA))
    f = np.concatenate([fi, fw])
    assert abs(e - e2) / abs(e) < 1e-13
    assert np.abs(w - w2).max() / abs(e) < 1e-13
    assert np.linalg.norm(f - f2) / np.linalg.norm(f) < 1e-13


def test_forces_are_energy_gradient(ewald, w64):
    pos, q = w64.all_pos(), w64.all_q()
    _, _, f = ewald.recip(pos, q, w64.box, BETA, KE)
    h = 1e-4
    rng = np.random.default_rng(7)
    for j in rng.choice(pos.shape[0], 6, replace=False):
        for a in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[j, a] += h
            p2[j, a] -= h
            e1, _, _ = ewald.recip(p1, q, w64.box, BETA, KE, forces=False)
            e2, _, _ = ewald.recip(p2, q, w64.box, BETA, KE, forces=False)
            fd = -(e1 - e2) / (2 * h)
            assert abs(fd - f[j, a]) <= 1e-8 * max(1.0, np.abs(f).max())


def test_zero_net_force(ewald, w64):
    _, _, f = ewald.recip(w64.all_pos(), w64.all_q(), w64.box, BETA, KE)
    frms = np.sqrt((f ** 2).mean())
    assert np.linalg.norm(f.sum(0)) / (math.sqrt(f.shape[0]) * frms) < 1e-12


def test_translation_invariance(ewald, w64):
    pos, q = w64.all_pos(), w64.all_q()
    e, w, f = ewald.recip(pos, q, w64.box, BETA, KE)
    shift = np.array([0.37, -1.91, 5.03])
    e2, w2, f2 = ewald.recip(np.mod(pos + shift, w64.box), q, w64.box, BETA, KE)
    assert abs(e2 - e) / abs(e) < 1e-12
    assert np.abs(w2 - w).max() / abs(e) < 1e-12
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 1e-12


def test_cutoff_converged(ewald, w64):
    pos, q = w64.all_pos(), w64.all_q()
    e, w, f = ewald.recip(pos, q, w64.box, BETA, KE)
    e2, w2, f2 = ewald.recip(pos, q, w64.box, BETA, KE, mcut=ewald.mcut_for(BETA, 1e-20))
    assert abs(e2 - e) / abs(e) < 1e-14
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 1e-14
    # the documented cutoff: exp(-pi^2 m^2/beta^2) = 1e-16 gives index radius ~10 at 12.42 A
    assert int(math.floor(ewald.mcut_for(BETA) * 12.42)) == 9


def test_k_count_matches_sphere(ewald):
    L = 49.7
    mc = ewald.mcut_for(BETA)
    nk = ewald.count_k([L, L, L], mc)
    expect = (4.0 / 3.0) * math.pi * (mc * L) ** 3 / 2
    assert abs(nk - expect) / expect < 0.02


def test_virial_diagonal_is_strain_derivative(ewald, w64):
    pos, q = w64.all_pos(), w64.all_q()
    _, w, _ = ewald.recip(pos, q, w64.box, BETA, KE, forces=False)
    d = 1e-6
    for a in range(3):
        s = np.ones(3)
        s[a] = 1 + d
        e1, _, _ = ewald.recip(pos * s, q, w64.box * s, BETA, KE, forces=False)
        s[a] = 1 - d
        e2, _, _ = ewald.recip(pos * s, q, w64.box * s, BETA, KE, forces=False)
        fd = -(e1 - e2) / (2 * d)
        assert abs(fd - w[a]) < 1e-7 * abs(w[a]) + 1e-9


def test_virial_offdiagonal_is_shear_derivative(ewald):
    # a small system keeps the twin's general-cell sum cheap
    s = systems.water_box(8, 7.0, seed=11)
    pos, q = s.all_pos(), s.all_q()
    mc = ewald.mcut_for(BETA)
    _, w, _ = ewald.recip(pos, q, s.box, BETA, KE, forces=False)
    d = 1e-6
    for idx, (a, b) in zip((3, 4, 5), ((0, 1), (0, 2), (1, 2))):
        es = []
        for sgn in (1, -1):
            F = np.eye(3)
            F[a, b] = sgn * d          # r_a += eps r_b
            es.append(ewald_np.recip_general(pos @ F.T, q, np.diag(s.box) @ F.T, BETA, KE, mc))
        fd = -(es[0] - es[1]) / (2 * d)
        assert abs(fd - w[idx]) < 1e-7 * np.abs(w).max()


def test_forces_on_subset_match_full(ewald, w64):
    pos, q = w64.all_pos(), w64.all_q()
    _, _, f = ewald.recip(pos, q, w64.box, BETA, KE)
    idx = np.array([5, 0, 200, 17])
    _, _, fs = ewald.recip(pos, q, w64.box, BETA, KE, force_idx=idx)
    assert np.array_equal(fs, f[idx])


def test_invalid_arguments_rejected(ewald):
    with pytest.raises(ValueError):
        ewald.recip(np.zeros((2, 3)), np.zeros(2), [0.0, 1.0, 1.0], BETA, KE)
    with pytest.raises(ValueError):
        ewald.recip(np.zeros((2, 3)), np.zeros(2), [1.0, 1.0, 1.0], BETA, KE, force_idx=[5])


def test_mesh_mode_restricted_forces(ewald):
    """recip_forces_mesh_modes: with a cube of modes that holds the whole
    converged sphere it is the full reciprocal sum (the C oracle); restricted
    to the modes of a 2.02 A mesh on the spacing-matched training box it misses
    Ewald by more than 1e-2 (the floor quoted for the learned coarse form)."""
    from oracle import ewald_np
    s = systems.workload(1).system()
    pos, q = s.all_pos(), s.all_q()
    _, _, F0 = ewald.recip(pos, q, s.box, systems.BETA, systems.COULOMB_K)
    nmax = int(np.ceil(ewald.mcut_for(systems.BETA) * s.box[0]))
    F1 = ewald_np.recip_forces_mesh_modes(pos, q, s.box, systems.BETA, systems.COULOMB_K, (2 * nmax + 2,) * 3)
    assert np.linalg.norm(F1 - F0) <= 1e-12 * np.linalg.norm(F0)
    t = systems.training_box(0)
    pos, q = t.all_pos(), t.all_q()
    _, _, Fe = ewald.recip(pos, q, t.box, systems.BETA, systems.COULOMB_K)
    Ft = ewald_np.recip_forces_mesh_modes(pos, q, t.box, systems.BETA, systems.COULOMB_K, (16, 16, 16))
    floor = np.linalg.norm(Ft - Fe) / np.linalg.norm(Fe)
    assert 1e-2 < floor < 2e-2
