"""What a correction on a 2x coarser mesh can reach: the numbers behind the
learned coarse form's feasibility, computed with the oracle only.

Systems: the spacing-matched training boxes (1,128 waters, 32.325 A, the
density of the 216k system), coarse mesh 16^3 (h = 2.02 A, the spacing of 64^3
on the 129.3 A box), order 5; the reference is the FP64 Ewald oracle.

  floor_mesh_modes   exact Ewald forces restricted to the modes a 16^3 mesh
                     holds, against full Ewald: the error left by any method
                     whose long-range part lives on the coarse mesh, with no
                     aliasing at all
  coarse_pppm        coarse-mesh PPPM against Ewald
  linear_<features>  coarse PPPM plus the best linear correction (ridge fit
                     on 8 training boxes, evaluated on 3 held-out boxes) in
                     rotation-equivariant vector features:
                       pair<rc>: q_i sum_j q_j g_k(r_ij) s(r_ij) rhat_ij,
                         Chebyshev radial basis within rc (translation
                         invariant; the kind of quantity the network's
                         descriptor is built from), per species of i;
                       self: q_i^2 times Fourier modes of the particle's
                         offset inside its coarse cell (mesh-relative)

Writes learned_floor.json next to this file; uses only oracle/ and systems/.
Run: python tests/golden/learned_floor.py (about 3 minutes on 8 cores).
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import systems  # noqa: E402
from oracle import ewald, ewald_np, learned as OL, pppm  # noqa: E402

KE, BETA = systems.COULOMB_K, systems.BETA
KC, P = 16, 5


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def box_data(i, heldout=False):
    s = systems.training_box(i, heldout)
    pos, q = s.all_pos(), s.all_q()
    _, Fc, _ = pppm.pppm(pos, q, s.box, (KC,) * 3, P, BETA, KE)
    _, _, Fe = ewald.recip(pos, q, s.box, BETA, KE)
    return s, pos, q, Fc, Fe


def pair_feats(pos, q, box, rc, nk):
    i, j, d = OL.neighbours(pos, box, rc)
    r = np.linalg.norm(d, axis=1)
    g = OL.chebyshev(2 * r / rc - 1, nk) * (0.5 * (1 + np.cos(math.pi * r / rc)))[:, None]
    u = d / r[:, None]
    V = np.zeros((pos.shape[0], nk, 3))
    np.add.at(V, i, (q[j][:, None] * g)[:, :, None] * u[:, None, :])
    return q[:, None, None] * V


def species_split(V, q):
    return np.concatenate([V * (q == qq)[:, None, None] for qq in (6.0, 1.0, -8.0)], axis=1)


def self_feats(pos, q, box):
    u = pos / (box / KC)
    d = u - np.floor(u)
    fs = []
    for m in (1, 2, 3):
        fs.append(np.sin(2 * math.pi * m * d))
        fs.append(np.cos(2 * math.pi * m * d))
    for m in (1, 2):
        for mp in (1, 2):
            c = np.cos(2 * math.pi * mp * d)
            fs.append(np.sin(2 * math.pi * m * d) * (c[:, [1, 2, 0]] + c[:, [2, 0, 1]]))
    return (q * q)[:, None, None] * np.stack(fs, axis=1)


def design(pos, q, box, sets):
    blocks = []
    for st in sets:
        if st[0] == "pair":
            blocks.append(species_split(pair_feats(pos, q, box, st[1], st[2]), q))
        else:
            blocks.append(species_split(self_feats(pos, q, box), q))
    return np.concatenate(blocks, axis=1)


def fit_eval(sets, ntrain=8, ntest=3, lam=1e-8):
    Xs, Ys = [], []
    for b in range(ntrain):
        s, pos, q, Fc, Fe = box_data(b)
        X = design(pos, q, s.box, sets)
        Xs.append(X.transpose(0, 2, 1).reshape(-1, X.shape[1]))
        Ys.append((Fe - Fc).reshape(-1))
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    sc = np.sqrt((X * X).mean(0)) + 1e-30
    A = X / sc
    w = np.linalg.solve(A.T @ A + lam * len(Y) * np.eye(A.shape[1]), A.T @ Y) / sc
    num = den = numc = 0.0
    for b in range(ntest):
        s, pos, q, Fc, Fe = box_data(b, heldout=True)
        pred = np.einsum("nfa,f->na", design(pos, q, s.box, sets), w)
        num += ((Fc + pred - Fe) ** 2).sum()
        numc += ((Fc - Fe) ** 2).sum()
        den += (Fe ** 2).sum()
    return math.sqrt(num / den), math.sqrt(numc / den), int(X.shape[1])


def main():
    ewald.build(force=False)
    out = {}
    s, pos, q, Fc, Fe = box_data(0)
    Ft = ewald_np.recip_forces_mesh_modes(pos, q, s.box, BETA, KE, (KC,) * 3)
    out["floor_mesh_modes"] = rel(Ft, Fe)
    out["coarse_pppm"] = rel(Fc, Fe)
    for name, sets in [("pair4", [("pair", 4.0, 32)]), ("pair6", [("pair", 6.0, 32)]),
                       ("pair8", [("pair", 8.0, 40)]), ("self", [("self",)]),
                       ("pair6+self", [("pair", 6.0, 32), ("self",)])]:
        e, ec, nf = fit_eval(sets)
        out[f"linear_{name}"] = {"rel_rmse_vs_ewald": e, "coarse_rel_rmse_vs_ewald": ec, "features": nf}
        print(name, out[f"linear_{name}"], flush=True)
    out["target"] = 1e-3
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_floor.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
