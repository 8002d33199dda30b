"""Closed-form and series solutions used to pin the oracle (test-side only).

None of this is the method under test: these are classical solutions of the
same boundary value problem (eq. BVP, sound-soft, v = -u_inc) that the MFS
scattering-matrix method must reproduce.

* disk_series          single sound-soft disk, Jacobi-Anger expansion
* mie_series           single sound-soft sphere, Mie (partial-wave) series
* MultiDisk            many sound-soft disks by the multipole method with
                       Graf's addition theorem (DLMF 10.23.7; P. A. Martin,
                       Multiple Scattering, 2006, ch. 4)
"""

from __future__ import annotations

import numpy as np
import scipy.special as sp


def disk_series(kappa, a, alpha, pts, centre=(0.0, 0.0), nmax=None):
    """u_s(r, th) = -sum_n i^n J_n(ka)/H_n(ka) H_n(kr) e^{i n (th - alpha)} for
    u_inc = exp(i kappa (cos alpha, sin alpha).x) and a disk of radius a."""
    c = np.asarray(centre, dtype=np.float64)
    rel = pts - c[None, :]
    r = np.hypot(rel[:, 0], rel[:, 1])
    th = np.arctan2(rel[:, 1], rel[:, 0])
    nmax = nmax or int(kappa * a + 40)
    u = np.zeros(pts.shape[0], dtype=np.complex128)
    phase0 = np.exp(1j * kappa * (np.cos(alpha) * c[0] + np.sin(alpha) * c[1]))
    for n in range(-nmax, nmax + 1):
        coef = -(1j ** n) * sp.jv(n, kappa * a) / sp.hankel1(n, kappa * a)
        u += coef * sp.hankel1(n, kappa * r) * np.exp(1j * n * (th - alpha))
    return phase0 * u


def mie_series(kappa, a, direction, pts, lmax=None):
    """u_s = -sum_l (2l+1) i^l j_l(ka)/h_l(ka) h_l(kr) P_l(cos gamma), h_l = j_l + i y_l."""
    d = np.asarray(direction, dtype=np.float64)
    r = np.linalg.norm(pts, axis=1)
    cg = (pts @ d) / r
    lmax = lmax or int(kappa * a + 40)
    u = np.zeros(pts.shape[0], dtype=np.complex128)
    for ell in range(lmax + 1):
        ha = sp.spherical_jn(ell, kappa * a) + 1j * sp.spherical_yn(ell, kappa * a)
        hr = sp.spherical_jn(ell, kappa * r) + 1j * sp.spherical_yn(ell, kappa * r)
        coef = -(2 * ell + 1) * (1j ** ell) * sp.spherical_jn(ell, kappa * a) / ha
        u += coef * hr * sp.eval_legendre(ell, cg)
    return u


class MultiDisk:
    """Sound-soft scattering by equal disks, multipole method.

    u_scat(x) = sum_j sum_{|n|<=nmax} c_{j,n} H_n(kappa |x - c_j|) e^{i n arg(x - c_j)}.
    With Graf's theorem H_n(k|x-c_j|)e^{in arg(x-c_j)} = sum_m H_{n-m}(k d)
    e^{i(n-m) psi} J_m(k rho) e^{i m theta} for x = c_l + rho e^{i theta},
    c_l - c_j = d e^{i psi}, rho < d, the boundary condition u_inc + u_scat = 0
    on |x - c_l| = a gives one equation per (l, m).
    """

    def __init__(self, kappa, a, centres, alpha, nmax=25):
        self.kappa, self.a, self.nmax = kappa, a, nmax
        self.centres = np.asarray(centres, dtype=np.float64)
        T = self.centres.shape[0]
        modes = np.arange(-nmax, nmax + 1)
        L = modes.size
        M = np.zeros((T * L, T * L), dtype=np.complex128)
        rhs = np.zeros(T * L, dtype=np.complex128)
        ka = kappa * a
        Jm = sp.jv(modes, ka)
        Hm = sp.hankel1(modes, ka)
        dvec = np.array([np.cos(alpha), np.sin(alpha)])
        for l in range(T):
            rows = slice(l * L, (l + 1) * L)
            M[rows, rows] += np.diag(Hm)
            rhs[rows] = -Jm * np.exp(1j * kappa * (dvec @ self.centres[l])) * (1j ** modes) * \
                np.exp(-1j * modes * alpha)
            for j in range(T):
                if j == l:
                    continue
                rel = self.centres[l] - self.centres[j]
                dist = np.hypot(*rel)
                psi = np.arctan2(rel[1], rel[0])
                diff = modes[None, :] - modes[:, None]  # n - m, rows m, cols n
                M[rows, j * L:(j + 1) * L] += Jm[:, None] * sp.hankel1(diff, kappa * dist) * \
                    np.exp(1j * diff * psi)
        self.coef = np.linalg.solve(M, rhs).reshape(T, L)
        self.modes = modes

    def field(self, pts):
        u = np.zeros(pts.shape[0], dtype=np.complex128)
        for j, c in enumerate(self.centres):
            rel = pts - c[None, :]
            r = np.hypot(rel[:, 0], rel[:, 1])
            th = np.arctan2(rel[:, 1], rel[:, 0])
            for n, cn in zip(self.modes, self.coef[j]):
                u += cn * sp.hankel1(n, self.kappa * r) * np.exp(1j * n * th)
        return u


def graf_check(kappa, n, cj, cl, x):
    """Both sides of Graf's addition theorem at one point (used to pin MultiDisk)."""
    rel = x - cj
    lhs = sp.hankel1(n, kappa * np.hypot(*rel)) * np.exp(1j * n * np.arctan2(rel[1], rel[0]))
    dl = cl - cj
    d, psi = np.hypot(*dl), np.arctan2(dl[1], dl[0])
    rr = x - cl
    rho, th = np.hypot(*rr), np.arctan2(rr[1], rr[0])
    m = np.arange(-60, 61)
    rhs = np.sum(sp.hankel1(n - m, kappa * d) * np.exp(1j * (n - m) * psi) * sp.jv(m, kappa * rho) *
                 np.exp(1j * m * th))
    return lhs, rhs
