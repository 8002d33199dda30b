"""The workloads, as seeded scene factories.

Each factory takes an optional body count T so that the same generator gives a
scaled-down scene for CPU checks (the box side is scaled to keep the body
density fixed).  Readings of unspecified parameters (proxy radius, equivalent
point radius, MFS offsets, counts) are the ones listed in the design notes:

* 16 disks: radius 1 on a 4x4 grid, spacing 3, kappa 5, m=128, n=64 at r=0.7,
  k=64 equivalent points at r=1.2, proxy circle r=1.5 with p=128; one plane
  wave at angle 0.
* 2000 starfish r(t)=0.5(1+0.3cos5t) in a 100x100 box (centre distance >= 1.5),
  kappa 10, m=256, n=128 (offset 0.06), k=128 on r=0.67, proxy r=0.75, p=257;
  one plane wave at a seeded angle.
* 1000 unit spheres in a 40^3 box (centre distance >= 3), kappa 3, m=900,
  n=400 on r=0.7, k=400 on r=1.2, proxy p=900 on r=1.5; direction (1,0,0).
* 2000 mixed bodies (disk, ellipse 1:0.5, starfish, kite; bounding radius 0.65)
  with k = 64/128/192/256 on r=0.70, m=2k, n=k, proxy r=0.75, p=m+1; kappa 20;
  R=64 plane waves at angles 2 pi r / 64.  MFS offset 0.06 inward, except the kite
  (0.03: its concave side has a small radius of curvature, and at 0.06 the
  single-body field error is 4e-6 against 2e-8 at 0.03).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .scenes import Scene, grid_centres_2d, plane_wave_directions_2d, random_centres
from .shapes import disk2d, ellipse2d, kite2d, sphere3d, starfish2d

BASE_SEED = 20260313


@dataclass(frozen=True)
class WorkloadConfig:
    key: str
    description: str
    dim: int
    kappa: float
    T: int
    R: int
    tol: float
    precision: str  # "fp64" or "mixed"


def c1_disks16(T: int = 16) -> Scene:
    side = int(round(np.sqrt(T)))
    if side * side != T:
        raise ValueError("the disk grid needs a square body count")
    shape = disk2d(radius=1.0, m=128, n=64, src_radius=0.7, k=64, rho_eq=1.2, p=128, r_psi=1.5)
    centres = grid_centres_2d(side, side, 3.0)
    return Scene(dim=2, kappa=5.0, shapes=[shape], shape_of=np.zeros(T, np.int32),
                 centres=centres, directions=plane_wave_directions_2d([0.0]),
                 name=f"disks{T}_kappa5")


def c2_starfish2000(T: int = 2000, seed: int = BASE_SEED + 1) -> Scene:
    shape = starfish2d(m=256, n=128, d=0.06, k=128, rho_eq=0.67, p=257, r_psi=0.75)
    box = 100.0 * np.sqrt(T / 2000.0)
    centres = random_centres(T, 2, box, 1.5, seed)
    rng = np.random.default_rng(seed + 7919)
    alpha = 2.0 * np.pi * rng.uniform()
    return Scene(dim=2, kappa=10.0, shapes=[shape], shape_of=np.zeros(T, np.int32),
                 centres=centres, directions=plane_wave_directions_2d([alpha]),
                 name=f"starfish{T}_kappa10")


def c3_spheres1000(T: int = 1000, seed: int = BASE_SEED + 2) -> Scene:
    shape = sphere3d(radius=1.0, m=900, n=400, src_radius=0.7, k=400, rho_eq=1.2, p=900,
                     r_psi=1.5)
    box = 40.0 * (T / 1000.0) ** (1.0 / 3.0)
    centres = random_centres(T, 3, box, 3.0, seed)
    return Scene(dim=3, kappa=3.0, shapes=[shape], shape_of=np.zeros(T, np.int32),
                 centres=centres, directions=np.array([[1.0, 0.0, 0.0]]),
                 name=f"spheres{T}_kappa3")


def c4_shapes():
    return [
        disk2d(radius=0.65, m=128, n=64, src_radius=0.455, k=64, rho_eq=0.70, p=129, r_psi=0.75),
        ellipse2d(a=0.65, b=0.325, m=256, n=128, d=0.06, k=128, rho_eq=0.70, p=257, r_psi=0.75),
        starfish2d(m=384, n=192, d=0.06, k=192, rho_eq=0.70, p=385, r_psi=0.75),
        kite2d(bounding=0.65, m=512, n=256, d=0.03, k=256, rho_eq=0.70, p=513, r_psi=0.75),
    ]


def c4_mixed_multi_incidence(T: int = 2000, R: int = 64, seed: int = BASE_SEED + 3) -> Scene:
    shapes = c4_shapes()
    box = 100.0 * np.sqrt(T / 2000.0)
    centres = random_centres(T, 2, box, 1.5, seed)
    rng = np.random.default_rng(seed + 104729)
    shape_of = rng.integers(0, len(shapes), size=T).astype(np.int32)
    angles = 2.0 * np.pi * np.arange(R) / R
    return Scene(dim=2, kappa=20.0, shapes=shapes, shape_of=shape_of, centres=centres,
                 directions=plane_wave_directions_2d(angles), name=f"mixed{T}_kappa20_R{R}")


CONFIGS = {
    "disks16": WorkloadConfig("disks16", "2D plain FP64, 16 disks, kappa 5", 2, 5.0, 16, 1,
                              1e-10, "fp64"),
    "starfish2000": WorkloadConfig("starfish2000", "2D 2000 starfish, kappa 10, FP32 matvec + "
                                   "FP64 GMRES-IR", 2, 10.0, 2000, 1, 1e-8, "mixed"),
    "spheres1000": WorkloadConfig("spheres1000", "3D 1000 spheres, kappa 3", 3, 3.0, 1000, 1,
                                  1e-8, "mixed"),
    "mixed2000_R64": WorkloadConfig("mixed2000_R64", "2D 2000 mixed bodies, kappa 20, R=64", 2,
                                    20.0, 2000, 64, 1e-8, "mixed"),
}


def make_scene(key: str, T: int | None = None) -> Scene:
    if key == "disks16":
        return c1_disks16(16 if T is None else T)
    if key == "starfish2000":
        return c2_starfish2000(2000 if T is None else T)
    if key == "spheres1000":
        return c3_spheres1000(1000 if T is None else T)
    if key == "mixed2000_R64":
        return c4_mixed_multi_incidence(2000 if T is None else T)
    raise KeyError(key)
