"""Writes the stored Ewald reference values used by the full-size GPU tests.

Calls only the oracle (oracle/ewald.c through oracle/ewald.py, and the PPPM
oracle oracle/pppm.py) on the seeded synthetic systems of the `systems`
package, at the FP32-rounded coordinates the FP32 kernels receive.  Output:
tests/golden/ewald_<workload>.json (FP64 Ewald) or
tests/golden/pppm_<workload>_<mesh>_p<order>.json (FP64 PPPM oracle) with the
energy, the virial and the forces on a seeded sample of particles.

    python tests/golden/make_golden.py [workload_index | fd | pppm:<index>:<mesh>:<order> ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import systems  # noqa: E402
from oracle import ewald, pppm  # noqa: E402

SAMPLE = 2048
SAMPLE_SEED = 4242


def make(k: int):
    w = systems.workload(k)
    s = w.system().rounded(np.float32)
    n = s.n
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=min(SAMPLE, n), replace=False))
    t = time.time()
    e, vir, f = ewald.recip(s.all_pos(), s.all_q(), s.box, w.beta, w.coulomb_k, force_idx=idx)
    dt = time.time() - t
    out = {
        "workload": w.name, "n_ion": s.n_ion, "n_wc": s.n_wc, "box": s.box.tolist(),
        "beta": w.beta, "coulomb_k": w.coulomb_k, "positions": "float32-rounded",
        "mcut": ewald.mcut_for(w.beta), "energy": e, "virial": vir.tolist(),
        "sample_seed": SAMPLE_SEED, "sample_index": idx.tolist(), "sample_force": f.tolist(),
        "oracle_seconds": dt, "oracle_threads": ewald.threads_used(),
        "generator": "tests/golden/make_golden.py (oracle/ewald.c, FP64 direct reciprocal sum)",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"ewald_{w.name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{path}: E={e:.12g} in {dt:.1f}s on {out['oracle_threads']} threads", flush=True)


FD_COUNT = 32
FD_SEED = 32
FD_STEP = 1e-4


def make_fd(k: int = 2):
    """Central finite differences (h = 1e-4 A) of the Ewald energy with respect
    to the coordinates of FD_COUNT seeded particles, plus the oracle's analytic
    forces on the same particles."""
    w = systems.workload(k)
    s = w.system().rounded(np.float32)
    pos, q = s.all_pos(), s.all_q()
    idx = np.sort(np.random.default_rng(FD_SEED).choice(s.n, FD_COUNT, replace=False))
    t = time.time()
    _, _, f = ewald.recip(pos, q, s.box, w.beta, w.coulomb_k, force_idx=idx)
    grad = np.zeros((FD_COUNT, 3))
    for i, j in enumerate(idx):
        for a in range(3):
            e = []
            for sg in (1, -1):
                p = pos.copy()
                p[j, a] += sg * FD_STEP
                e.append(ewald.recip(p, q, s.box, w.beta, w.coulomb_k, forces=False)[0])
            grad[i, a] = (e[0] - e[1]) / (2 * FD_STEP)
    out = {"workload": w.name, "positions": "float32-rounded", "step": FD_STEP, "seed": FD_SEED,
           "index": idx.tolist(), "fd_gradient": grad.tolist(), "oracle_force": f.tolist(),
           "oracle_seconds": time.time() - t,
           "generator": "tests/golden/make_golden.py fd (oracle/ewald.c energies)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"ewald_fd_{w.name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{path}: {time.time() - t:.1f}s", flush=True)


def make_pppm(k: int, mesh: int, order: int, alias: int = 2):
    """FP64 PPPM oracle (ik differentiation, alias range |m| <= alias) at mesh^3:
    energy, virial and the forces on the same seeded sample as make()."""
    w = systems.workload(k)
    s = w.system().rounded(np.float32)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(s.n, size=min(SAMPLE, s.n), replace=False))
    t = time.time()
    e, f, vir = pppm.pppm(s.all_pos(), s.all_q(), s.box, (mesh,) * 3, order, w.beta, w.coulomb_k, alias)
    dt = time.time() - t
    out = {
        "workload": w.name, "n_ion": s.n_ion, "n_wc": s.n_wc, "box": s.box.tolist(),
        "beta": w.beta, "coulomb_k": w.coulomb_k, "positions": "float32-rounded",
        "mesh": mesh, "order": order, "alias": alias, "energy": e, "virial": np.asarray(vir).tolist(),
        "sample_seed": SAMPLE_SEED, "sample_index": idx.tolist(), "sample_force": f[idx].tolist(),
        "oracle_seconds": dt,
        "generator": "tests/golden/make_golden.py pppm (oracle/pppm.py, FP64 PPPM-ik)",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"pppm_{w.name}_{mesh}_p{order}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{path}: E={e:.12g} in {dt:.1f}s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:] or ["3"]
    for a in args:
        if a == "fd":
            make_fd(2)
        elif a.startswith("pppm:"):
            _, k, mesh, order = a.split(":")
            make_pppm(int(k), int(mesh), int(order))
        else:
            make(int(a))
