"""Seeded request streams for the serving loop (inputs only).

Each request is a scattering scene drawn from a fixed ten-shape library: dimension 2 or 3, a body count
log-uniform in [t_min, t_max], shapes uniform from the dimension's library, a wavenumber from the
dimension's list, 1..r_max incident directions, and a Poisson arrival time.  Body density matches the
starfish (2D) and sphere (3D) workloads.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .scenes import Scene, plane_wave_directions_2d, random_centres
from .shapes import cshape2d, disk2d, ellipse2d, ellipsoid3d, kite2d, rod2d, sphere3d, starfish2d, teardrop2d, torus3d


def shape_library_2d():
    """Seven 2D shapes of bounding radius 0.65 (k = 64..256 equivalent points), two of them with
    corners and the rod with its cap junctions (Gauss-Legendre panels refined toward them)."""
    return {
        "disk": disk2d(radius=0.65, m=128, n=64, src_radius=0.455, k=64, rho_eq=0.70, p=129, r_psi=0.75),
        "ellipse": ellipse2d(a=0.65, b=0.325, m=256, n=128, d=0.06, k=128, rho_eq=0.70, p=257, r_psi=0.75),
        "starfish": starfish2d(m=256, n=128, d=0.06, k=128, rho_eq=0.67, p=257, r_psi=0.75),
        "kite": kite2d(bounding=0.65, m=512, n=256, d=0.03, k=256, rho_eq=0.70, p=513, r_psi=0.75),
        "teardrop": teardrop2d(levels=8, base_panels=16, d_frac=0.5, k=128),
        "cshape": cshape2d(levels=6, base_per_edge=3, d_frac=0.5, k=128),
        "rod": rod2d(levels=4, k=128),
    }


def shape_library_3d():
    """Three 3D shapes (k = 400) resolved for kappa <= 5."""
    return {
        "sphere": sphere3d(radius=1.0, m=900, n=400, src_radius=0.7, k=400, rho_eq=1.2, p=900, r_psi=1.5),
        "ellipsoid": ellipsoid3d(axes=(1.0, 0.75, 0.5), m=900, n=400, src_scale=0.7, k=400, p=900),
        "torus": torus3d(n_u=40, n_v=20, k=400, p=900),
    }


KAPPAS = {2: (5.0, 10.0, 20.0), 3: (3.0, 5.0)}


@dataclass
class RequestSpec:
    rid: int
    arrival: float
    scene: Scene
    shape_keys: list = field(default_factory=list)
    geometry: int = -1          # requests with equal ids share bodies, shapes and wavenumber


def _directions(rng, dim: int, R: int) -> np.ndarray:
    if dim == 2:
        return plane_wave_directions_2d(2.0 * np.pi * rng.uniform(size=R))
    d = rng.normal(size=(R, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def request_stream(n: int, rate: float, seed: int, t_min: int = 4, t_max: int = 64, r_max: int = 16,
                   p3d: float = 0.5, p_sweep: float = 0.0) -> list:
    """n requests with exponential inter-arrival times of mean 1/rate (seconds).  With probability
    p_sweep a request revisits the geometry of an earlier one with new incident directions (an
    incidence sweep over one configuration); such requests can share a solve."""
    rng = np.random.default_rng(seed)
    lib = {2: shape_library_2d(), 3: shape_library_3d()}
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        if out and p_sweep > 0.0 and rng.uniform() < p_sweep:
            base = out[int(rng.integers(len(out)))]
            R = int(rng.integers(1, r_max + 1))
            b = base.scene
            sc = Scene(dim=b.dim, kappa=b.kappa, shapes=b.shapes, shape_of=b.shape_of, centres=b.centres,
                       directions=_directions(rng, b.dim, R),
                       name=f"req{rid}_d{b.dim}_T{b.T}_k{b.kappa:g}_R{R}_g{base.geometry}")
            out.append(RequestSpec(rid=rid, arrival=t, scene=sc, shape_keys=base.shape_keys, geometry=base.geometry))
            continue
        dim = 3 if rng.uniform() < p3d else 2
        T = int(round(np.exp(rng.uniform(np.log(t_min), np.log(t_max)))))
        keys = list(lib[dim].keys())
        shape_of = rng.integers(0, len(keys), size=T).astype(np.int32)
        kappa = float(rng.choice(KAPPAS[dim]))
        R = int(rng.integers(1, r_max + 1))
        if dim == 2:
            box = 100.0 * np.sqrt(T / 2000.0)
            centres = random_centres(T, 2, max(box, 1.6), 1.5, int(rng.integers(1 << 30)))
        else:
            box = 40.0 * (T / 1000.0) ** (1.0 / 3.0)
            centres = random_centres(T, 3, max(box, 3.2), 3.0, int(rng.integers(1 << 30)))
        dirs = _directions(rng, dim, R)
        sc = Scene(dim=dim, kappa=kappa, shapes=[lib[dim][k] for k in keys], shape_of=shape_of,
                   centres=centres, directions=dirs, name=f"req{rid}_d{dim}_T{T}_k{kappa:g}_R{R}")
        out.append(RequestSpec(rid=rid, arrival=t, scene=sc, shape_keys=keys, geometry=rid))
    return out
