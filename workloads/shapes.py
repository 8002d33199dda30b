"""Point sets for one scatterer shape (geometry only, float64).

Every shape is described in its own body frame (reference point at the
origin).  A discretisation carries the four point sets the method needs
(Sec. 3.2-3.4 and Sec. 4.1-4.2 of the paper):

* ``colloc`` -- m collocation points x_i on the boundary Gamma,
* ``src``    -- n MFS sources y_j inside Gamma, on a curve a distance d in
  from Gamma along the inward normal (Sec. 3.2: n = m/2 in 2D),
* ``proxy``  -- p proxy points z_i on the proxy surface Psi enclosing Gamma,
* ``eqpts``  -- k equivalent-source points x_hat, where incoming fields are
  sampled and outgoing fields are represented.

All arrays are point-major ``[count, dim]``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class ShapeDiscretisation:
    name: str
    dim: int
    colloc: np.ndarray
    src: np.ndarray
    proxy: np.ndarray
    eqpts: np.ndarray
    bounding_radius: float
    proxy_radius: float
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.colloc.shape[0]

    @property
    def n(self) -> int:
        return self.src.shape[0]

    @property
    def p(self) -> int:
        return self.proxy.shape[0]

    @property
    def k(self) -> int:
        return self.eqpts.shape[0]


def circle_points(count: int, radius: float, offset: float = 0.0) -> np.ndarray:
    """``count`` points equispaced in angle on a circle about the origin."""
    t = 2.0 * np.pi * (np.arange(count, dtype=np.float64) + offset) / count
    return np.stack([radius * np.cos(t), radius * np.sin(t)], axis=-1)


def fibonacci_sphere(count: int, radius: float) -> np.ndarray:
    """Fibonacci lattice on a sphere: z_i = 1-(2i+1)/k, azimuth i*pi*(3-sqrt5)."""
    i = np.arange(count, dtype=np.float64)
    zc = 1.0 - (2.0 * i + 1.0) / count
    s = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    az = i * np.pi * (3.0 - np.sqrt(5.0))
    return radius * np.stack([s * np.cos(az), s * np.sin(az), zc], axis=-1)


# --------------------------------------------------------------------------
# 2D parametrised curves: each returns (points, outward unit normals) at the
# parameter values t.
# --------------------------------------------------------------------------

def _polar_curve(t, f, fp):
    """Curve (f(t) cos t, f(t) sin t) with derivative f'(t)."""
    c, s = np.cos(t), np.sin(t)
    pts = np.stack([f * c, f * s], axis=-1)
    tan = np.stack([fp * c - f * s, fp * s + f * c], axis=-1)
    return pts, tan


def _normals_from_tangent(tan):
    # counter-clockwise curve: outward normal is the tangent rotated by -90 deg
    nrm = np.stack([tan[:, 1], -tan[:, 0]], axis=-1)
    return nrm / np.linalg.norm(nrm, axis=1)[:, None]


def _curve_points(kind: str, t: np.ndarray, params: dict):
    if kind == "disk":
        a = params["radius"]
        f = np.full_like(t, a)
        fp = np.zeros_like(t)
        pts, tan = _polar_curve(t, f, fp)
    elif kind == "starfish":
        r0, amp, lobes = params["r0"], params["amp"], params["lobes"]
        f = r0 * (1.0 + amp * np.cos(lobes * t))
        fp = -r0 * amp * lobes * np.sin(lobes * t)
        pts, tan = _polar_curve(t, f, fp)
    elif kind == "ellipse":
        a, b = params["a"], params["b"]
        pts = np.stack([a * np.cos(t), b * np.sin(t)], axis=-1)
        tan = np.stack([-a * np.sin(t), b * np.cos(t)], axis=-1)
    elif kind == "kite":
        sc = params["scale"]
        pts = sc * np.stack([np.cos(t) + 0.65 * np.cos(2 * t) - 0.65, 1.5 * np.sin(t)], axis=-1)
        tan = sc * np.stack([-np.sin(t) - 1.3 * np.sin(2 * t), 1.5 * np.cos(t)], axis=-1)
    else:
        raise ValueError(f"unknown 2D shape kind {kind!r}")
    return pts, _normals_from_tangent(tan)


def _discretise_curve(name, kind, params, m, n, d, k, rho_eq, p, r_psi, bounding):
    t_col = 2.0 * np.pi * np.arange(m, dtype=np.float64) / m
    t_src = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    colloc, _ = _curve_points(kind, t_col, params)
    on_curve, nrm = _curve_points(kind, t_src, params)
    src = on_curve - d * nrm  # inward along the normal (Sec. 3.2)
    return ShapeDiscretisation(
        name=name,
        dim=2,
        colloc=colloc,
        src=src,
        proxy=circle_points(p, r_psi),
        eqpts=circle_points(k, rho_eq),
        bounding_radius=bounding,
        proxy_radius=r_psi,
        meta=dict(kind=kind, params=params, d=d, rho_eq=rho_eq),
    )


def disk2d(radius=1.0, m=128, n=64, src_radius=0.7, k=64, rho_eq=1.2, p=128, r_psi=1.5):
    """Disk of the given radius; MFS sources on a concentric circle."""
    return _discretise_curve("disk", "disk", dict(radius=radius), m, n, radius - src_radius,
                             k, rho_eq, p, r_psi, radius)


def starfish2d(m=256, n=128, d=0.06, k=128, rho_eq=0.67, p=257, r_psi=0.75,
               r0=0.5, amp=0.3, lobes=5):
    """Starfish r(theta) = r0 (1 + amp cos(lobes theta)); bounding radius r0(1+amp)."""
    return _discretise_curve("starfish", "starfish", dict(r0=r0, amp=amp, lobes=lobes),
                             m, n, d, k, rho_eq, p, r_psi, r0 * (1.0 + amp))


def ellipse2d(a=0.65, b=0.325, m=256, n=128, d=0.06, k=128, rho_eq=0.70, p=257, r_psi=0.75):
    return _discretise_curve("ellipse", "ellipse", dict(a=a, b=b), m, n, d, k, rho_eq, p,
                             r_psi, max(a, b))


def kite2d(bounding=0.65, m=512, n=256, d=0.02, k=256, rho_eq=0.70, p=513, r_psi=0.75):
    """The classical inverse-scattering kite, rescaled to the given bounding radius.  Its wing tips
    are sharply curved: sources much deeper than d = 0.02 fold over there and the MFS fit stalls
    near 1e-3 (d = 0.06) or 2e-5 (d = 0.03) on the boundary, against 8e-6 at d = 0.02."""
    t = np.linspace(0.0, 2.0 * np.pi, 4097)
    raw = np.stack([np.cos(t) + 0.65 * np.cos(2 * t) - 0.65, 1.5 * np.sin(t)], axis=-1)
    scale = bounding / np.linalg.norm(raw, axis=1).max()
    return _discretise_curve("kite", "kite", dict(scale=scale), m, n, d, k, rho_eq, p,
                             r_psi, bounding)


# --------------------------------------------------------------------------
# 3D surfaces: Fibonacci point sets mapped radially onto the surface.
# --------------------------------------------------------------------------

def _radial_surface(name, radius_fn, m, n, src_scale, k, rho_eq, p, r_psi, bounding, meta):
    u_col = fibonacci_sphere(m, 1.0)
    u_src = fibonacci_sphere(n, 1.0)
    colloc = u_col * radius_fn(u_col)[:, None]
    src = u_src * (src_scale * radius_fn(u_src))[:, None]
    return ShapeDiscretisation(
        name=name,
        dim=3,
        colloc=colloc,
        src=src,
        proxy=fibonacci_sphere(p, r_psi),
        eqpts=fibonacci_sphere(k, rho_eq),
        bounding_radius=bounding,
        proxy_radius=r_psi,
        meta=dict(meta, src_scale=src_scale, rho_eq=rho_eq),
    )


def sphere3d(radius=1.0, m=900, n=400, src_radius=0.7, k=400, rho_eq=1.2, p=900, r_psi=1.5):
    """Sphere with Fibonacci collocation, MFS sources, proxy and equivalent points."""
    return _radial_surface("sphere", lambda u: np.full(u.shape[0], radius), m, n,
                           src_radius / radius, k, rho_eq, p, r_psi, radius,
                           dict(kind="sphere", radius=radius))


def ellipsoid3d(axes=(1.0, 0.75, 0.5), m=900, n=400, src_scale=0.7, k=400, p=900):
    ax = np.asarray(axes, dtype=np.float64)

    def rad(u):
        return 1.0 / np.sqrt(((u / ax) ** 2).sum(-1))

    b = float(ax.max())
    return _radial_surface("ellipsoid", rad, m, n, src_scale, k, 1.2 * b, p, 1.5 * b, b,
                           dict(kind="ellipsoid", axes=tuple(axes)))


def bumpy_sphere3d(m=900, n=400, src_scale=0.7, k=400, p=900):
    """r = 1 + 0.1 cos(3 theta) sin(2 phi) in spherical angles."""

    def rad(u):
        th = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
        ph = np.arctan2(u[:, 1], u[:, 0])
        return 1.0 + 0.1 * np.cos(3 * th) * np.sin(2 * ph)

    return _radial_surface("bumpy_sphere", rad, m, n, src_scale, k, 1.32, p, 1.65, 1.1,
                           dict(kind="bumpy_sphere"))


# --------------------------------------------------------------------------
# Curves with corners: Gauss-Legendre panels, dyadically refined toward the
# corners, MFS sources offset in proportion to each panel's length.
# --------------------------------------------------------------------------

def _teardrop_raw(t, beta):
    """Teardrop (2 sin(t/2), -beta sin t): one corner at t = 0, counter-clockwise."""
    pts = np.stack([2.0 * np.sin(0.5 * t), -beta * np.sin(t)], axis=-1)
    der = np.stack([np.cos(0.5 * t), -beta * np.cos(t)], axis=-1)
    return pts, der


def _panel_breaks(base_panels: int, levels: int) -> np.ndarray:
    """Panel end points in [0, 2 pi]: base_panels equal panels, the two next to the corner at
    t = 0 = 2 pi split dyadically `levels` times toward it."""
    h = 2.0 * np.pi / base_panels
    inner = list(np.linspace(h, 2.0 * np.pi - h, base_panels - 1))
    near0 = [h / 2.0 ** l for l in range(levels, 0, -1)]
    near2pi = [2.0 * np.pi - x for x in reversed(near0)]
    return np.array([0.0] + near0 + inner + near2pi + [2.0 * np.pi])


def teardrop2d(bounding=0.65, beta=1.0, base_panels=16, levels=8, q=16, d_frac=0.2, k=128, rho_eq=0.70,
               r_psi=0.75, p=None):
    """Teardrop with a corner, scaled to the given bounding radius (centred on its bounding box).

    Each panel carries q Gauss-Legendre collocation points and q/2 MFS sources (n = m/2), the
    sources offset inward by d_frac times the panel's arclength.  Equivalent points: k on a circle
    of radius rho_eq (the paper-mode skeleton can be taken from the collocation points instead).
    """
    breaks = _panel_breaks(base_panels, levels)
    xq, _ = np.polynomial.legendre.leggauss(q)
    xs, _ = np.polynomial.legendre.leggauss(q // 2)
    col_t, src_t, src_d = [], [], []
    # arclength of each panel from a fine quadrature of |gamma'|
    xg, wg = np.polynomial.legendre.leggauss(32)
    for a, b in zip(breaks[:-1], breaks[1:]):
        mid, half = 0.5 * (a + b), 0.5 * (b - a)
        _, dg = _teardrop_raw(mid + half * xg, beta)
        length = half * float(np.sum(wg * np.linalg.norm(dg, axis=1)))
        col_t.append(mid + half * xq)
        src_t.append(mid + half * xs)
        src_d.append(np.full(q // 2, d_frac * length))
    col_t, src_t, src_d = np.concatenate(col_t), np.concatenate(src_t), np.concatenate(src_d)
    raw_c, _ = _teardrop_raw(col_t, beta)
    raw_s, der_s = _teardrop_raw(src_t, beta)
    # centre and scale from a fixed dense sampling of the exact curve, so that every
    # discretisation describes the same body
    dense, _ = _teardrop_raw(np.linspace(0.0, 2.0 * np.pi, 200001), beta)
    lo, hi = dense.min(0), dense.max(0)
    centre = 0.5 * (lo + hi)
    scale = bounding / np.linalg.norm(dense - centre, axis=1).max()
    colloc = (raw_c - centre) * scale
    on_curve = (raw_s - centre) * scale
    tang = der_s / np.linalg.norm(der_s, axis=1, keepdims=True)
    outward = np.stack([tang[:, 1], -tang[:, 0]], axis=-1)  # counter-clockwise curve
    src = on_curve - (src_d * scale)[:, None] * outward
    m = colloc.shape[0]
    return ShapeDiscretisation(
        name="teardrop", dim=2, colloc=colloc, src=src,
        proxy=circle_points(p if p is not None else m + 1, r_psi),
        eqpts=circle_points(k, rho_eq), bounding_radius=bounding, proxy_radius=r_psi,
        meta=dict(kind="teardrop", beta=beta, base_panels=base_panels, levels=levels, q=q, d_frac=d_frac,
                  corner=(np.array([0.0, 0.0]) - centre) * scale))


def _polygon_panels(vertices, base_per_edge, levels, q, d_frac):
    """Collocation points and MFS sources on a counter-clockwise polygon: each edge is split into
    base_per_edge panels, the end panels refined dyadically toward both vertices; q Gauss-Legendre
    collocation points and q/2 sources per panel, sources offset inward along the edge normal by
    d_frac times the panel length."""
    xq, _ = np.polynomial.legendre.leggauss(q)
    xs, _ = np.polynomial.legendre.leggauss(q // 2)
    col, src = [], []
    V = np.asarray(vertices, np.float64)
    for e in range(V.shape[0]):
        a, b = V[e], V[(e + 1) % V.shape[0]]
        edge = b - a
        length = float(np.linalg.norm(edge))
        tang = edge / length
        inward = np.array([-tang[1], tang[0]])  # left of the direction of travel
        h = 1.0 / base_per_edge
        brk = [0.0] + [h / 2.0 ** l for l in range(levels, 0, -1)]
        brk += list(np.linspace(h, 1.0 - h, base_per_edge - 1))
        brk += [1.0 - h / 2.0 ** l for l in range(1, levels + 1)] + [1.0]
        brk = np.array(sorted(set(brk)))
        for s0, s1 in zip(brk[:-1], brk[1:]):
            mid, half = 0.5 * (s0 + s1), 0.5 * (s1 - s0)
            plen = 2.0 * half * length
            col.append(a[None, :] + (mid + half * xq)[:, None] * edge[None, :])
            src.append(a[None, :] + (mid + half * xs)[:, None] * edge[None, :] + d_frac * plen * inward[None, :])
    return np.concatenate(col), np.concatenate(src)


def cshape2d(bounding=0.65, base_per_edge=4, levels=8, q=16, d_frac=0.5, k=128, rho_eq=0.70, r_psi=0.75,
             p=None):
    """A C-shaped cavity (a square with a slot cut into one side): eight corners, two of them
    re-entrant, scaled to the given bounding radius."""
    raw = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, -0.3], [-0.3, -0.3], [-0.3, 0.3], [1.0, 0.3],
                    [1.0, 1.0], [-1.0, 1.0]])
    scale = bounding / np.linalg.norm(raw, axis=1).max()
    colloc, src = _polygon_panels(raw * scale, base_per_edge, levels, q, d_frac)
    m = colloc.shape[0]
    return ShapeDiscretisation(
        name="cshape", dim=2, colloc=colloc, src=src, proxy=circle_points(p if p is not None else m + 1, r_psi),
        eqpts=circle_points(k, rho_eq), bounding_radius=bounding, proxy_radius=r_psi,
        meta=dict(kind="cshape", base_per_edge=base_per_edge, levels=levels, q=q, d_frac=d_frac,
                  vertices=raw * scale))


def _rod_pieces(a, r):
    """The four pieces of a rod (a 2a x 2r rectangle with semicircular caps of radius r),
    counter-clockwise: each maps s in [0, 1] to (points, inward unit normals), with its length."""
    def bottom(s):
        pts = np.stack([-a + 2.0 * a * s, np.full_like(s, -r)], axis=-1)
        return pts, np.tile([0.0, 1.0], (s.size, 1))

    def top(s):
        pts = np.stack([a - 2.0 * a * s, np.full_like(s, r)], axis=-1)
        return pts, np.tile([0.0, -1.0], (s.size, 1))

    def cap(cx, th0):
        def f(s):
            th = th0 + np.pi * s
            out = np.stack([np.cos(th), np.sin(th)], axis=-1)
            return np.array([cx, 0.0])[None, :] + r * out, -out
        return f

    return [(bottom, 2.0 * a), (cap(a, -0.5 * np.pi), np.pi * r), (top, 2.0 * a), (cap(-a, 0.5 * np.pi), np.pi * r)]


def rod2d(bounding=0.65, aspect=6.0, base_per_side=8, base_per_cap=4, levels=6, q=16, d_frac=0.5, k=128,
          rho_eq=0.70, r_psi=0.75, p=None):
    """A rod: a thin rectangle with semicircular caps (Sec. 5.1 Example 4), length 2 bounding and
    thickness 2 bounding / aspect.  The curvature jumps where the caps meet the sides, so every
    piece is split into Gauss-Legendre panels refined dyadically toward both of its ends, with q
    collocation points and q/2 MFS sources per panel, the sources offset inward by d_frac times the
    panel length (less than the cap radius)."""
    r = bounding / aspect
    a = bounding - r
    xq, _ = np.polynomial.legendre.leggauss(q)
    xs, _ = np.polynomial.legendre.leggauss(q // 2)
    col, src = [], []
    for piece, length in _rod_pieces(a, r):
        base = base_per_side if piece.__name__ in ("bottom", "top") else base_per_cap
        h = 1.0 / base
        brk = [0.0] + [h / 2.0 ** l for l in range(levels, 0, -1)]
        brk += list(np.linspace(h, 1.0 - h, base - 1))
        brk += [1.0 - h / 2.0 ** l for l in range(1, levels + 1)] + [1.0]
        brk = np.array(sorted(set(brk)))
        for s0, s1 in zip(brk[:-1], brk[1:]):
            mid, half = 0.5 * (s0 + s1), 0.5 * (s1 - s0)
            plen = 2.0 * half * length
            pc, _ = piece(mid + half * xq)
            ps, nin = piece(mid + half * xs)
            col.append(pc)
            src.append(ps + min(d_frac * plen, 0.5 * r) * nin)
    colloc, src = np.concatenate(col), np.concatenate(src)
    m = colloc.shape[0]
    return ShapeDiscretisation(
        name="rod", dim=2, colloc=colloc, src=src, proxy=circle_points(p if p is not None else m + 1, r_psi),
        eqpts=circle_points(k, rho_eq), bounding_radius=bounding, proxy_radius=r_psi,
        meta=dict(kind="rod", half_length=a, radius=r, base_per_side=base_per_side, base_per_cap=base_per_cap,
                  levels=levels, q=q, d_frac=d_frac,
                  junctions=np.array([[-a, -r], [a, -r], [a, r], [-a, r]])))


def torus3d(R0=0.7, a=0.3, n_u=40, n_v=20, src_frac=0.3, k=400, rho_eq=None, p=900, r_psi=None):
    """Torus ((R0 + a cos v) cos u, (R0 + a cos v) sin u, a sin v) on a tensor grid in (u, v)
    (Sec. 3.4): n_u x n_v collocation points, (n_u/2) x (n_v/2) MFS sources (n = m/4) on the
    concentric torus of tube radius src_frac * a.  Equivalent and proxy points on spheres about
    the centre (a torus is not star-shaped, but both spheres enclose it)."""
    def grid(nu, nv, tube):
        u = 2.0 * np.pi * (np.arange(nu) + 0.5) / nu
        v = 2.0 * np.pi * (np.arange(nv) + 0.5) / nv
        U, V = np.meshgrid(u, v, indexing="ij")
        rr = R0 + tube * np.cos(V)
        return np.stack([rr * np.cos(U), rr * np.sin(U), tube * np.sin(V)], -1).reshape(-1, 3)
    bounding = R0 + a
    rho = 1.2 * bounding if rho_eq is None else rho_eq
    rp = 1.5 * bounding if r_psi is None else r_psi
    return ShapeDiscretisation(
        name="torus", dim=3, colloc=grid(n_u, n_v, a), src=grid(n_u // 2, n_v // 2, src_frac * a),
        proxy=fibonacci_sphere(p, rp), eqpts=fibonacci_sphere(k, rho), bounding_radius=bounding,
        proxy_radius=rp, meta=dict(kind="torus", R0=R0, a=a, n_u=n_u, n_v=n_v, src_frac=src_frac))
