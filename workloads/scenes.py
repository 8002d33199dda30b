"""Seeded body placements, incident directions and field targets.

A scene is a list of shape templates plus, for each body tau, the index of its
shape and its centre c_tau.  Bodies of one shape are translated copies, so they
share one scattering matrix (the paper notes the matrix depends only on the
shape, Sec. 5.1 Example 4).  Packing the equivalent points of all bodies into
one global array is left to the consumers (oracle and library each do it).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .shapes import ShapeDiscretisation


@dataclass
class Scene:
    dim: int
    kappa: float
    shapes: list  # list[ShapeDiscretisation]
    shape_of: np.ndarray  # int32 [T]
    centres: np.ndarray  # float64 [T, dim]
    directions: np.ndarray  # float64 [R, dim], unit incident directions
    name: str = ""
    rotations: np.ndarray | None = None  # float64 [T, dim, dim] body orientations, None: identity

    def place(self, t: int, pts: np.ndarray) -> np.ndarray:
        """Body-frame points of body t in world coordinates: R_t p + c_t."""
        if self.rotations is None:
            return pts + self.centres[t][None, :]
        return pts @ self.rotations[t].T + self.centres[t][None, :]

    @property
    def T(self) -> int:
        return int(self.shape_of.shape[0])

    @property
    def R(self) -> int:
        return int(self.directions.shape[0])

    @property
    def k_of_shape(self) -> np.ndarray:
        return np.array([s.k for s in self.shapes], dtype=np.int64)

    @property
    def N(self) -> int:
        return int(self.k_of_shape[self.shape_of].sum())

    def n_pairs(self) -> int:
        """Off-body pair count per matvec: N^2 - sum_tau k_tau^2."""
        k = self.k_of_shape[self.shape_of].astype(np.int64)
        return int(k.sum() ** 2 - (k * k).sum())

    def radius(self) -> float:
        c = self.centres
        mid = 0.5 * (c.min(0) + c.max(0))
        rb = max(s.bounding_radius for s in self.shapes)
        return float(np.linalg.norm(c - mid, axis=1).max() + rb)

    def middle(self) -> np.ndarray:
        return 0.5 * (self.centres.min(0) + self.centres.max(0))


def grid_centres_2d(nx: int, ny: int, spacing: float) -> np.ndarray:
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    return np.stack([spacing * i.ravel(), spacing * j.ravel()], axis=-1).astype(np.float64)


def random_centres(count: int, dim: int, box: float, min_dist: float, seed: int,
                   max_tries: int = 200000) -> np.ndarray:
    """Uniform centres in [0, box]^dim with pairwise distance >= min_dist.

    Sequential rejection sampling with a cell hash; deterministic for a seed.
    """
    rng = np.random.default_rng(seed)
    cell = min_dist
    ncell = max(1, int(np.ceil(box / cell)))
    grid: dict = {}
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries * max(1, count // 100 + 1):
            raise RuntimeError("could not place bodies: box too crowded")
        c = rng.uniform(0.0, box, size=dim)
        key = tuple(np.minimum((c // cell).astype(int), ncell - 1))
        ok = True
        for off in np.ndindex(*([3] * dim)):
            nb = tuple(key[a] + off[a] - 1 for a in range(dim))
            for other in grid.get(nb, ()):
                if np.sum((out[other] - c) ** 2) < min_dist * min_dist:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            grid.setdefault(key, []).append(len(out))
            out.append(c)
    return np.asarray(out, dtype=np.float64)


def plane_wave_directions_2d(angles) -> np.ndarray:
    a = np.asarray(angles, dtype=np.float64).reshape(-1)
    return np.stack([np.cos(a), np.sin(a)], axis=-1)


def far_targets(scene: Scene, count: int = 64, factor: float = 2.0) -> np.ndarray:
    """Targets on a circle (2D) or Fibonacci sphere (3D) of radius factor x scene radius."""
    rad = factor * scene.radius()
    mid = scene.middle()
    if scene.dim == 2:
        t = 2.0 * np.pi * (np.arange(count) + 0.25) / count
        pts = np.stack([np.cos(t), np.sin(t)], axis=-1)
    else:
        from .shapes import fibonacci_sphere

        pts = fibonacci_sphere(count, 1.0)
    return mid[None, :] + rad * pts


def shapes_summary(shapes: list) -> str:
    return ", ".join(f"{s.name}(m={s.m},n={s.n},p={s.p},k={s.k})" for s in shapes)


__all__ = [
    "Scene",
    "ShapeDiscretisation",
    "grid_centres_2d",
    "random_centres",
    "plane_wave_directions_2d",
    "far_targets",
    "shapes_summary",
]


def random_rotations(T: int, dim: int, seed: int) -> np.ndarray:
    """T seeded proper rotations: angles uniform in 2D, uniform on SO(3) in 3D (QR of a Gaussian
    matrix with the sign fixed)."""
    rng = np.random.default_rng(seed)
    if dim == 2:
        a = rng.uniform(0.0, 2.0 * np.pi, size=T)
        c, s = np.cos(a), np.sin(a)
        return np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)
    out = np.empty((T, 3, 3))
    for t in range(T):
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out[t] = q
    return out
