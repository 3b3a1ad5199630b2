"""Seeded synthetic inputs (geometry only) shared by the oracle tests, the GPU
tests and the benchmark.  Nothing here computes electrostatics."""
from .water import (System, water_box, ionic_box, displaced_frames, nacl_crystal,
                    COULOMB_K, BETA, SEED_BASE)
from .configs import WORKLOADS, Workload, workload, training_box

__all__ = ["System", "water_box", "ionic_box", "displaced_frames", "nacl_crystal",
           "COULOMB_K", "BETA", "SEED_BASE", "WORKLOADS", "Workload", "workload",
           "training_box"]
