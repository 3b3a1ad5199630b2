"""The seeded input generators: determinism and the stated geometry."""
import math

import numpy as np

import systems
from systems import water


def test_seeded_and_deterministic():
    a = systems.workload(2).system()
    b = systems.workload(2).system()
    assert np.array_equal(a.ion_pos, b.ion_pos) and np.array_equal(a.wc_pos, b.wc_pos)
    c = systems.water_box(4096, 49.7, seed=1)
    assert not np.array_equal(a.ion_pos, c.ion_pos)


def _unwrap(d, L):
    return d - L * np.round(d / L)


def test_water_geometry_and_charges():
    s = systems.workload(2).system()
    L = s.box
    o, h1, h2 = s.ion_pos[0::3], s.ion_pos[1::3], s.ion_pos[2::3]
    d1, d2 = _unwrap(h1 - o, L), _unwrap(h2 - o, L)
    assert np.allclose(np.linalg.norm(d1, axis=1), 0.96, atol=1e-12)
    assert np.allclose(np.linalg.norm(d2, axis=1), 0.96, atol=1e-12)
    ang = np.degrees(np.arccos((d1 * d2).sum(1) / 0.96 ** 2))
    assert np.allclose(ang, 104.5, atol=1e-9)
    dw = _unwrap(s.wc_pos - o, L)
    assert np.allclose(np.linalg.norm(dw, axis=1), 0.25, atol=1e-12)
    bis = (d1 + d2) / np.linalg.norm(d1 + d2, axis=1, keepdims=True)
    assert np.allclose((dw / 0.25 * bis).sum(1), 1.0, atol=1e-12)
    assert abs(s.all_q().sum()) == 0.0
    assert set(np.unique(s.ion_q)) == {1.0, 6.0} and set(np.unique(s.wc_q)) == {-8.0}
    pos = s.all_pos()
    assert (pos >= 0).all() and (pos < L).all()


def test_workload_sizes():
    w3 = systems.workload(3)
    s = w3.system()
    assert (s.n_ion, s.n_wc) == (216576, 72192)
    assert abs(72192 / 129.3 ** 3 - water.WATER_DENSITY) < 2e-4
    assert w3.n_particles == 288768


def test_displaced_frames():
    s = systems.workload(1).system()
    fr = list(systems.displaced_frames(s, 3, 0.02, seed=5))
    assert np.array_equal(fr[0].ion_pos, s.ion_pos)
    d = _unwrap(fr[1].ion_pos - fr[0].ion_pos, s.box)
    assert 0.015 < d.std() < 0.025


def test_ionic_min_distance():
    s = systems.ionic_box(500, 10, 26.0, seed=3)
    from scipy.spatial import cKDTree
    ions = s.ion_pos[1500:]
    assert ions.shape[0] == 20
    tree = cKDTree(ions, boxsize=26.0)
    others = np.concatenate([s.ion_pos[:1500], s.wc_pos])
    o_idx = np.arange(0, 1500, 3)
    not_o = np.ones(others.shape[0], bool)
    not_o[o_idx] = False                 # lattice-site oxygens keep the lattice spacing
    d, _ = tree.query(others[not_o], k=1)
    assert d.min() >= 2.5
    assert abs(s.all_q().sum()) < 1e-12


def test_training_box_spacing_matched():
    t = systems.training_box(0)
    assert t.n_wc == 1128 and abs(t.box[0] * 4 - 129.3) < 1e-12
