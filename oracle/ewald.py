"""Python front end of the FP64 C Ewald oracle (oracle/ewald.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the GPU product path.

The oracle evaluates the DPLR Gaussian-charge energy E_Gt (DPLR background
section: the reciprocal sum over m != 0 of exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2
divided by 2 pi V, with S(m) running over ions and Wannier centroids) times the
Coulomb constant, its forces and its virial, by the direct sum over k-vectors.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald.c")
_LIB = os.path.join(_HERE, "libewald_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_ewald_recip.argtypes = [i64, p, p, p, d, d, d, p, p, i64, p, p]
        lib.oracle_ewald_recip.restype = ctypes.c_int
        lib.oracle_ewald_real.argtypes = [i64, p, p, p, d, d, d, p, p]
        lib.oracle_ewald_real.restype = ctypes.c_int
        lib.oracle_ewald_self.argtypes = [i64, p, d, d]
        lib.oracle_ewald_self.restype = d
        lib.oracle_count_k.argtypes = [p, d]
        lib.oracle_count_k.restype = i64
        lib.oracle_threads_used.argtypes = []
        lib.oracle_threads_used.restype = i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def mcut_for(beta: float, tol: float = 1e-16) -> float:
    """Reciprocal cutoff |m| with exp(-pi^2 m^2 / beta^2) = tol."""
    return beta * math.sqrt(math.log(1.0 / tol)) / math.pi


def count_k(box, mcut: float) -> int:
    box = np.ascontiguousarray(box, dtype=np.float64)
    return int(_load().oracle_count_k(_ptr(box), mcut))


def threads_used() -> int:
    return int(_load().oracle_threads_used())


def recip(pos, q, box, beta: float, ke: float, mcut: Optional[float] = None,
          force_idx=None, forces: bool = True, tol: float = 1e-16):
    """Reciprocal Ewald energy, virial (xx,yy,zz,xy,xz,yz) and forces.

    pos [n,3], q [n], box [3].  force_idx: indices of the particles whose forces
    are wanted (None = all when forces is True).  Returns (E, W[6], F[k,3])."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    if mcut is None:
        mcut = mcut_for(beta, tol)
    n = pos.shape[0]
    e = np.zeros(1)
    w = np.zeros(6)
    if forces:
        idx = np.arange(n, dtype=np.int64) if force_idx is None else \
            np.ascontiguousarray(force_idx, dtype=np.int64)
        f = np.zeros((idx.shape[0], 3))
        rc = _load().oracle_ewald_recip(n, _ptr(pos), _ptr(q), _ptr(box), beta, ke, mcut,
                                        _ptr(e), _ptr(w), idx.shape[0], _ptr(idx), _ptr(f))
    else:
        f = np.zeros((0, 3))
        rc = _load().oracle_ewald_recip(n, _ptr(pos), _ptr(q), _ptr(box), beta, ke, mcut,
                                        _ptr(e), _ptr(w), 0, None, None)
    if rc != 0:
        raise ValueError(f"oracle_ewald_recip failed with status {rc}")
    return float(e[0]), w, f


def real(pos, q, box, beta: float, ke: float, rcut: Optional[float] = None, tol: float = 1e-17):
    """Real-space Ewald energy and forces over images within rcut."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    if rcut is None:
        # erfc(x) < tol for x > sqrt(ln(1/tol)) (a loose upper bound)
        rcut = math.sqrt(math.log(1.0 / tol)) / beta
    e = np.zeros(1)
    f = np.zeros_like(pos)
    rc = _load().oracle_ewald_real(pos.shape[0], _ptr(pos), _ptr(q), _ptr(box), beta, ke, rcut,
                                   _ptr(e), _ptr(f))
    if rc != 0:
        raise ValueError(f"oracle_ewald_real failed with status {rc}")
    return float(e[0]), f


def self_energy(q, beta: float, ke: float) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    return float(_load().oracle_ewald_self(q.shape[0], _ptr(q), beta, ke))


def full_energy(pos, q, box, beta: float, ke: float) -> float:
    """Total point-charge Coulomb energy of a neutral periodic system
    (tin-foil boundary) = reciprocal + real - self."""
    er, _, _ = recip(pos, q, box, beta, ke, forces=False)
    ed, _ = real(pos, q, box, beta, ke)
    return er + ed + self_energy(q, beta, ke)


def system_recip(sys, beta: float, ke: float, force_idx=None, forces: bool = True,
                 mcut: Optional[float] = None):
    """recip() on a systems.System; forces split into (ion, wc) when all are asked."""
    pos, q = sys.all_pos(), sys.all_q()
    e, w, f = recip(pos, q, sys.box, beta, ke, mcut=mcut, force_idx=force_idx, forces=forces)
    if forces and force_idx is None:
        return e, w, f[: sys.n_ion], f[sys.n_ion:]
    return e, w, f
