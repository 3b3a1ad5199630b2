"""Seeded synthetic water / ionic-solution systems.

These generators build the inputs of the DPLR long-range step: ion (atom)
positions and charges plus Wannier-centroid (WC) positions and charges in a
periodic orthorhombic box.  The paper measures on liquid water where each WC is
bound to an oxygen atom (Evaluation section; the WC binding W_n = R_i + Delta_n
of the DPLR background section).  Its DFT water data set is not available, so
every workload here is synthetic: rigid water geometry on a jittered lattice,
random orientations, drawn with NumPy's PCG64 from a fixed seed.

This module holds geometry only (no electrostatics) and is shared by the
oracle-side tests and the GPU-side tests and benchmark.

Recipe (one water):
  * O on a jittered simple-cubic lattice (sigma = 0.1 A per coordinate);
  * O-H = 0.96 A, H-O-H = 104.5 degrees, orientation a uniform random rotation;
  * WC 0.25 A from O along the H-O-H bisector, on the hydrogen side;
  * charges O +6, H +1, WC -8 (a neutral molecule).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

OH_BOND = 0.96          # Angstrom
HOH_ANGLE_DEG = 104.5
WC_OFFSET = 0.25        # Angstrom from O along the bisector
Q_O, Q_H, Q_WC = 6.0, 1.0, -8.0
Q_NA, Q_CL = 1.0, -1.0
WATER_DENSITY = 0.0334  # molecules per cubic Angstrom
COULOMB_K = 14.399645   # eV * Angstrom / e^2
BETA = 0.4              # 1/Angstrom
SEED_BASE = 20260000


@dataclasses.dataclass
class System:
    """A periodic system: atoms ("ions") and Wannier centroids.

    ion_pos [n_ion, 3] float64 in [0, L), ion_q [n_ion];
    wc_pos [n_wc, 3] float64 in [0, L), wc_q [n_wc];
    box [3] float64 (orthorhombic edge lengths, Angstrom).
    """
    ion_pos: np.ndarray
    ion_q: np.ndarray
    wc_pos: np.ndarray
    wc_q: np.ndarray
    box: np.ndarray
    name: str = ""

    @property
    def n_ion(self) -> int:
        return int(self.ion_pos.shape[0])

    @property
    def n_wc(self) -> int:
        return int(self.wc_pos.shape[0])

    @property
    def n(self) -> int:
        return self.n_ion + self.n_wc

    def all_pos(self) -> np.ndarray:
        return np.concatenate([self.ion_pos, self.wc_pos], axis=0)

    def all_q(self) -> np.ndarray:
        return np.concatenate([self.ion_q, self.wc_q], axis=0)

    def rounded(self, dtype) -> "System":
        """Copy whose positions and charges are rounded to `dtype` and promoted
        back to float64, so a reference evaluated on it sees exactly the
        coordinates a reduced-precision kernel sees."""
        f = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)
        return System(f(self.ion_pos), f(self.ion_q), f(self.wc_pos), f(self.wc_q),
                      self.box.copy(), self.name)


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly distributed rotation matrices (unit quaternions drawn by
    Shoemake's subgroup method), shape [n, 3, 3]."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    w = a * np.sin(2 * np.pi * u2)
    x = a * np.cos(2 * np.pi * u2)
    y = b * np.sin(2 * np.pi * u3)
    z = b * np.cos(2 * np.pi * u3)
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def _molecule_frame() -> np.ndarray:
    """Body-frame offsets from O of (H1, H2, WC), shape [3, 3]; the bisector is +z."""
    half = math.radians(HOH_ANGLE_DEG) / 2
    h1 = [OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]
    h2 = [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]
    wc = [0.0, 0.0, WC_OFFSET]
    return np.array([h1, h2, wc])


def lattice_sites(n_sites: int, box: float, rng: np.random.Generator, jitter: float = 0.1):
    """Jittered simple-cubic lattice with m = ceil(n^(1/3)) sites per axis;
    when m^3 > n, a seeded permutation picks which n sites are kept."""
    m = int(math.ceil(round(n_sites ** (1.0 / 3.0), 9)))
    while m ** 3 < n_sites:
        m += 1
    a = box / m
    g = np.arange(m)
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3) * a + a / 2
    if m ** 3 > n_sites:
        keep = np.sort(rng.permutation(m ** 3)[:n_sites])
        sites = sites[keep]
    sites = sites + rng.normal(0.0, jitter, size=sites.shape)
    return sites, a


def _place_waters(o_pos: np.ndarray, rot: np.ndarray):
    frame = _molecule_frame()                      # [3, 3]
    off = np.einsum("nij,kj->nki", rot, frame)     # [n, 3(H1,H2,WC), 3]
    h1 = o_pos + off[:, 0]
    h2 = o_pos + off[:, 1]
    wc = o_pos + off[:, 2]
    return h1, h2, wc


def _wrap(p: np.ndarray, box: np.ndarray) -> np.ndarray:
    p = np.mod(p, box)
    # a tiny negative coordinate can round to exactly L; it belongs at 0
    return np.where(p >= box, 0.0, p)


def water_box(n_waters: int, box_len: float, seed: int, jitter: float = 0.1,
              name: str = "") -> System:
    """n_waters rigid waters in a cubic box of edge box_len (Angstrom)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    o_pos, _ = lattice_sites(n_waters, box_len, rng, jitter)
    rot = _random_rotations(rng, n_waters)
    h1, h2, wc = _place_waters(o_pos, rot)
    box = np.full(3, float(box_len))
    ion = np.stack([o_pos, h1, h2], axis=1).reshape(-1, 3)
    ion_q = np.tile([Q_O, Q_H, Q_H], n_waters).astype(np.float64)
    wc_q = np.full(n_waters, Q_WC)
    return System(_wrap(ion, box), ion_q, _wrap(wc, box), wc_q, box, name)


def ionic_box(n_waters: int, n_pairs: int, box_len: float, seed: int, jitter: float = 0.1,
              min_dist: float = 2.5, max_redraw: int = 200, name: str = "") -> System:
    """Waters plus n_pairs Na+ and n_pairs Cl- on lattice sites.  Any water with a
    particle closer than min_dist to an ion gets its orientation redrawn."""
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    n_sites = n_waters + 2 * n_pairs
    sites, _ = lattice_sites(n_sites, box_len, rng, jitter)
    perm = rng.permutation(n_sites)
    ion_sites = sites[perm[: 2 * n_pairs]]
    o_pos = sites[np.sort(perm[2 * n_pairs:])]
    box = np.full(3, float(box_len))
    rot = _random_rotations(rng, n_waters)
    ions_w = _wrap(ion_sites.copy(), box)
    tree = cKDTree(ions_w, boxsize=box_len)
    todo = np.arange(n_waters)
    for _ in range(max_redraw):
        h1, h2, wc = _place_waters(o_pos[todo], rot[todo])
        bad = np.zeros(len(todo), bool)
        for p in (h1, h2, wc):
            d, _ = tree.query(_wrap(p.copy(), box), k=1)
            bad |= d < min_dist
        if not bad.any():
            break
        todo = todo[bad]
        rot[todo] = _random_rotations(rng, len(todo))
    h1, h2, wc = _place_waters(o_pos, rot)
    water_ions = np.stack([o_pos, h1, h2], axis=1).reshape(-1, 3)
    ion = np.concatenate([water_ions, ion_sites], axis=0)
    ion_q = np.concatenate([np.tile([Q_O, Q_H, Q_H], n_waters),
                            np.full(n_pairs, Q_NA), np.full(n_pairs, Q_CL)]).astype(np.float64)
    return System(_wrap(ion, box), ion_q, _wrap(wc, box), np.full(n_waters, Q_WC), box, name)


def displaced_frames(sys0: System, n_frames: int, sigma: float, seed: int):
    """Cumulative random walk: frame t+1 = wrap(frame t + N(0, sigma^2)) on every
    coordinate of every particle (ions and WCs alike).  Yields Systems."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ion, wc = sys0.ion_pos.copy(), sys0.wc_pos.copy()
    for t in range(n_frames):
        yield System(ion.copy(), sys0.ion_q, wc.copy(), sys0.wc_q, sys0.box, f"{sys0.name}/frame{t}")
        ion = _wrap(ion + rng.normal(0.0, sigma, ion.shape), sys0.box)
        wc = _wrap(wc + rng.normal(0.0, sigma, wc.shape), sys0.box)


def nacl_crystal(cells: int = 2, a: float = 5.64) -> System:
    """Rock-salt crystal, `cells`^3 conventional cells of edge a; Na+ and Cl-
    are returned as ions (no WCs)."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    na, cl = [], []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                c = np.array([i, j, k], float)
                na.append((fcc + c) * a)
                cl.append((fcc + c + np.array([.5, 0, 0])) * a)
    pos = np.concatenate([np.concatenate(na), np.concatenate(cl)])
    q = np.concatenate([np.full(4 * cells ** 3, 1.0), np.full(4 * cells ** 3, -1.0)])
    box = np.full(3, cells * a)
    return System(_wrap(pos, box), q, np.zeros((0, 3)), np.zeros(0), box, f"nacl{cells}")
