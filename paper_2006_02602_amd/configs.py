"""Workload definitions: seeded synthetic cavities shaped like the paper's runs.

The paper times its buoyancy-driven-cavity code on 256^3 meshes at Ra = 1e5
(Sec. 2; Tables 3-4), meshes 32^3..1024^3, with 1D/2D/3D decompositions
(Sec. 3.2).  There is no dataset: every input is the seeded initial state of
include/cavity.h (fluid at rest up to +-noise, T linear between the walls).
"""
from dataclasses import dataclass
from typing import Tuple

from . import Grid, Halo, Params

CONFIG_WIDTHS = (1, 2, 2, 2, 2)    # p 1 layer; u, v, w, T 2 layers
PAPER_WIDTHS = (2, 1, 1, 1, 1)     # stencil-based widths of "Optimized V2" (Listing 2)


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    Ra: float
    steps: int
    seed: int
    splits: Tuple[Tuple[int, int, int], ...]
    widths: Tuple[int, int, int, int, int] = CONFIG_WIDTHS
    noise: float = 1e-3

    @property
    def grid(self) -> Grid:
        return Grid.cube(self.n)

    @property
    def params(self) -> Params:
        return Params(Ra=self.Ra, Pr=0.71, cfl=0.5)

    def halo(self, split=None, widths=None) -> Halo:
        return Halo(split or self.splits[0], widths or self.widths)


# small parity case: 16^3, Ra 1e3, 100 steps, 2x2x2 virtual split every step
C0 = Workload("cavity16_f64_ra1e3", 16, 1e3, 100, 1, ((2, 2, 2),))
# one GPU's share at the paper's size: 256^3, Ra 1e5, 200 steps; the headline
# step exchanges the 3D (2,2,2) split; 1D (8,1,1) and 2D (4,2,1) are timed too
C1 = Workload("cavity256_f64_ra1e5", 256, 1e5, 200, 2, ((2, 2, 2), (8, 1, 1), (4, 2, 1)))

WORKLOADS = {w.name: w for w in (C0, C1)}


# ---- batched form: 96 independent cubes of uneven sizes and Rayleigh numbers
_MASK = (1 << 64) - 1
BATCH_EDGES = (24, 32, 48, 64, 96)


def splitmix64(seed: int, n: int) -> int:
    """Output number n (0-based) of the SplitMix64 stream seeded with `seed`
    (Steele, Lea & Flood 2014)."""
    z = (seed + (n + 1) * 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def batch_workload(count: int = 96, seed: int = 4):
    """[(edge, Ra, init_seed)] of the batched workload: cube edges drawn
    uniformly from BATCH_EDGES and log10(Ra) uniformly from [3, 6] with
    SplitMix64(seed) outputs 2c and 2c+1 for cavity c; every cavity is seeded
    like the small parity case (noise 1e-3, T linear in x)."""
    out = []
    for c in range(count):
        edge = BATCH_EDGES[splitmix64(seed, 2 * c) % len(BATCH_EDGES)]
        r = (splitmix64(seed, 2 * c + 1) >> 11) * 2.0 ** -53
        out.append((edge, 10.0 ** (3.0 + 3.0 * r), seed * 1000 + c))
    return out


# ---- discrete adjoint: gradient of the hot-wall Nusselt number ------------
@dataclass(frozen=True)
class AdjointWorkload:
    """64^3 FP64 at Ra 1e4, 400 steps, checkpoints every 20; hot-wall
    temperatures 1 + 0.05 (2r - 1) with r from SplitMix64(seed) output
    j + nj k (53-bit uniform); initial state seeded like the parity case."""
    name: str = "adjoint64_f64_ra1e4"
    n: int = 64
    Ra: float = 1e4
    steps: int = 400
    every: int = 20
    seed: int = 5
    amp: float = 0.05

    @property
    def grid(self) -> Grid:
        return Grid.cube(self.n)

    def theta(self):
        import numpy as np
        nj = nk = self.n
        r = np.array([(splitmix64(self.seed, m) >> 11) * 2.0 ** -53 for m in range(nj * nk)])
        return 1.0 + self.amp * (2.0 * r - 1.0)


ADJOINT = AdjointWorkload()
