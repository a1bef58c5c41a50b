"""Named synthetic workloads (shapes and input recipes only, no exchange arithmetic).

Each workload stands in for a condensed-phase system of the paper
(Computational Details: 32-128 H2O boxes, Fe3+ in 64 H2O).  Grids are cubic;
``box`` is in bohr; ``kernel`` is 0 (spherically truncated Coulomb) or 1
(erfc-screened, parameter w in bohr^-1).

Seeds follow seed = 20230901 + 100 * k + system_index for workload k = 1..5.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import generate

TRUNCATED = 0
ERFC = 1


@dataclass(frozen=True)
class System:
    name: str
    n: int            # grid points per axis (cubic grid n^3)
    L: float          # cubic box length, bohr
    n_orb: int
    kernel: int
    param: float      # erfc w; ignored for the truncated kernel
    family: str       # "random_pw" or "gaussians"
    ecut: float       # band limit |G|^2/2 <= ecut, Hartree
    seed: int

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    @property
    def box(self):
        return (self.L, self.L, self.L)

    @property
    def n_pairs(self):
        return self.n_orb * (self.n_orb + 1) // 2

    def orbitals(self, n_orb=None):
        """Raw (normalised, not orthonormalised) float64 orbitals [orb, z, y, x]."""
        k = self.n_orb if n_orb is None else n_orb
        if self.family == "random_pw":
            return generate.random_pw(self.shape, self.box, k, self.ecut, self.seed)
        if self.family == "gaussians":
            return generate.gaussians(self.shape, self.box, k, self.ecut, self.seed)[0]
        raise ValueError(self.family)


def _seed(k, idx=0):
    return 20230901 + 100 * k + idx


# 1: plain FP64 method, tiny: random PW (5 Ha), truncated Coulomb.
TINY24 = System("tiny24", 24, 10.0, 8, TRUNCATED, 0.0, "random_pw", 5.0, _seed(1))

# 2: 64-water-like box: localised Gaussians (20 Ha), erfc w = 0.106.
WATER96 = System("water96", 96, 23.5, 256, ERFC, 0.106, "gaussians", 20.0, _seed(2))

# 3: six uneven boxes at constant grid spacing h = 23.5/96 bohr, random PW
#    orbitals as in workload 1, truncated Coulomb.
BATCHED6 = tuple(
    System(f"batched6.{i}", n, 23.5 * n / 96.0, no, TRUNCATED, 0.0, "random_pw", 5.0,
           _seed(3, i))
    for i, (no, n) in enumerate([(64, 64), (128, 72), (192, 80), (256, 96),
                                 (320, 108), (384, 120)]))

# 4: autograd workload: localised Gaussians (20 Ha), erfc w = 0.106.
GRAD72 = System("grad72", 72, 17.6, 128, ERFC, 0.106, "gaussians", 20.0, _seed(4))

# 5: large condensed-phase box: localised Gaussians (20 Ha), truncated Coulomb.
LARGE128 = System("large128", 128, 29.6, 512, TRUNCATED, 0.0, "gaussians", 20.0,
                  _seed(5))

ALL = {s.name: s for s in (TINY24, WATER96, GRAD72, LARGE128) + BATCHED6}
