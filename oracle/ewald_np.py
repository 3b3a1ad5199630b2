"""NumPy twin of the C Ewald oracle, for small systems (a few hundred charges).

TEST INFRASTRUCTURE ONLY.  It enumerates the FULL k sphere (both m and -m)
instead of the C code's doubled half space, and evaluates the phases
exp(2 pi i m.r) as one matrix, so the two oracles share neither code nor
summation structure.  Definitions as in the DPLR background section: the
energy is k_e/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2.
"""
from __future__ import annotations

import math

import numpy as np


def kvectors(box, mcut: float) -> np.ndarray:
    """All m = n / L with 0 < |m| <= mcut, shape [nk, 3]."""
    box = np.asarray(box, dtype=np.float64)
    nmax = np.floor(mcut * box).astype(int)
    g = [np.arange(-nmax[a], nmax[a] + 1) for a in range(3)]
    n = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    m = n / box
    m2 = (m * m).sum(1)
    keep = (m2 > 0) & (m2 <= mcut * mcut)
    return m[keep]


def recip(pos, q, box, beta: float, ke: float, mcut: float):
    """Returns (E, W[6], F[n,3]) by the plain full-sphere sum."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    m = kvectors(box, mcut)                           # [nk, 3]
    m2 = (m * m).sum(1)
    f = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2   # [nk]
    ph = np.exp(2j * math.pi * (pos @ m.T))           # [n, nk]
    S = q @ ph                                        # [nk]
    s2 = (S.conj() * S).real
    pre = ke / (2 * math.pi * V)
    E = pre * float((f * s2).sum())
    c = 2 * (1 + math.pi ** 2 * m2 / beta ** 2) / m2
    W = np.empty(6)
    for i, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        W[i] = pre * float((f * s2 * ((1.0 if a == b else 0.0) - c * m[:, a] * m[:, b])).sum())
    im = (S.conj()[None, :] * ph).imag                # [n, nk]
    F = (2 * ke / V) * q[:, None] * ((im * f[None, :]) @ m)
    return E, W, F


def recip_general(pos, q, hmat, beta: float, ke: float, mcut: float):
    """Energy for a general (triclinic) cell whose ROWS are the box vectors:
    m runs over n @ inv(h).T with 0 < |m| <= mcut.  Used to take strain
    derivatives in every direction."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    h = np.asarray(hmat, dtype=np.float64)
    V = abs(float(np.linalg.det(h)))
    hinvT = np.linalg.inv(h).T
    lens = np.linalg.norm(h, axis=1)
    nmax = np.ceil(mcut * lens * 1.05).astype(int) + 1
    g = [np.arange(-nmax[a], nmax[a] + 1) for a in range(3)]
    n = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    m = n @ hinvT
    m2 = (m * m).sum(1)
    keep = (m2 > 0) & (m2 <= mcut * mcut)
    m, m2 = m[keep], m2[keep]
    f = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2
    S = q @ np.exp(2j * math.pi * (pos @ m.T))
    return ke / (2 * math.pi * V) * float((f * (S.conj() * S).real).sum())


def recip_forces_mesh_modes(pos, q, box, beta: float, ke: float, K):
    """Reciprocal forces of the E_Gt sum restricted to the wave vectors a mesh
    of K[a] points per axis holds: m = n / L with 0 < |n_a| <= K[a] / 2 on every
    axis (the cube of mesh modes, not a sphere).  With K large enough to hold
    every mode of weight above rounding it is the full sum; for a coarse mesh
    it is the best any method limited to that mesh's modes can do, with no
    aliasing or assignment error."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    g = [np.arange(-(int(K[a]) // 2), int(K[a]) // 2 + 1) for a in range(3)]
    n = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    m = n / box
    m2 = (m * m).sum(1)
    keep = m2 > 0
    m, m2 = m[keep], m2[keep]
    f = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2
    ph = np.exp(2j * math.pi * (pos @ m.T))
    S = q @ ph
    im = (S.conj()[None, :] * ph).imag
    return (2 * ke / V) * q[:, None] * ((im * f[None, :]) @ m)
