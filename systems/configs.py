"""The five named workloads (seeded) and the learned-form training boxes.

Sizes follow the paper's water benchmark scaled to one GPU: the 216,576-atom
system is the atom count of the (8,6,8)-replicated 188-water base box of the
weak-scaling experiment (Evaluation, weak scaling), here rebuilt at liquid-water
density with 72,192 WCs.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

from .water import System, water_box, ionic_box, SEED_BASE, COULOMB_K, BETA


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_waters: int
    box: float
    mesh: int
    order: int
    precision: str              # "fp64" or "fp32"
    n_pairs: int = 0            # Na+/Cl- pairs (ionic solution)
    coarse_mesh: Optional[int] = None
    beta: float = BETA
    coulomb_k: float = COULOMB_K
    seed: int = 0

    def system(self) -> System:
        if self.n_pairs:
            return ionic_box(self.n_waters, self.n_pairs, self.box, self.seed, name=self.name)
        return water_box(self.n_waters, self.box, self.seed, name=self.name)

    @property
    def n_particles(self) -> int:
        return 4 * self.n_waters + 2 * self.n_pairs


WORKLOADS = {
    1: Workload("water64_fp64", 64, 12.42, 32, 5, "fp64", seed=SEED_BASE + 1),
    2: Workload("water4096_fp32", 4096, 49.7, 64, 5, "fp32", seed=SEED_BASE + 2),
    3: Workload("water72192_fp32", 72192, 129.3, 128, 5, "fp32", seed=SEED_BASE + 3),
    4: Workload("water72192_learned64", 72192, 129.3, 128, 5, "fp32", coarse_mesh=64,
                seed=SEED_BASE + 3),
    5: Workload("ionic306000_fp32", 300000, 208.5, 256, 5, "fp32", n_pairs=3000,
                coarse_mesh=128, seed=SEED_BASE + 5),
}


def workload(k: int) -> Workload:
    return WORKLOADS[k]


# Spacing-matched training boxes for the learned coarse-mesh form: the same
# water recipe and density as the 72,192-water system, on a box one quarter of
# its edge (1,128 waters in 32.325 A), so that meshes 16^3 / 32^3 there have the
# spacings of 64^3 / 128^3 on the full box.
TRAIN_WATERS = 1128
TRAIN_BOX = 129.3 / 4
TRAIN_SEED_BASE = SEED_BASE + 100000
HELDOUT_SEED_BASE = SEED_BASE + 200000


def training_box(i: int, heldout: bool = False) -> System:
    seed = (HELDOUT_SEED_BASE if heldout else TRAIN_SEED_BASE) + i
    return water_box(TRAIN_WATERS, TRAIN_BOX, seed, name=f"train{i}")
