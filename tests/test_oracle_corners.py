"""Pins for bodies with corners (Sec. 3.3: Gauss-Legendre panels, dyadic refinement toward the
corners, MFS distance scaled with the panel length).

There is no closed form for these shapes, so the pins are the ones the mathematics fixes: the
far field converges as the corner refinement deepens, the sound-soft boundary condition is met
between the collocation points away from the corners, and the scattering matrix (either mode)
reproduces the plain MFS solution it compresses.
"""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from oracle.fundamental import phi_matrix

KAPPA = 10.0
D0 = np.array([np.cos(0.3), np.sin(0.3)])
FAR = w.circle_points(48, 3.0, 0.1)


def _mfs_far_field(sh):
    A = phi_matrix(sh.colloc, sh.src, KAPPA)
    q = local_s.tsvd_solve(A, -np.exp(1j * KAPPA * sh.colloc @ D0), 1e-13)
    return phi_matrix(FAR, sh.src, KAPPA) @ q, q


@pytest.mark.parametrize("make,levels", [
    (lambda L: w.teardrop2d(levels=L, base_panels=32, d_frac=0.5), (6, 10, 14)),
    (lambda L: w.cshape2d(levels=L, base_per_edge=4, d_frac=0.5), (6, 8, 10)),
])
def test_far_field_converges_with_corner_refinement(make, levels):
    fields = [_mfs_far_field(make(L))[0] for L in levels]
    d1 = np.abs(fields[0] - fields[2]).max() / np.abs(fields[2]).max()
    d2 = np.abs(fields[1] - fields[2]).max() / np.abs(fields[2]).max()
    assert d2 < 0.3 * d1          # deeper refinement moves the answer less
    assert d2 < 1e-4              # measured: teardrop 4e-7, C-shape 3e-5


@pytest.mark.parametrize("make", [lambda: w.teardrop2d(levels=12, base_panels=32, d_frac=0.5),
                                  lambda: w.cshape2d(levels=10, base_per_edge=4, d_frac=0.5)])
def test_boundary_condition_between_collocation_points(make):
    sh = make()
    _, q = _mfs_far_field(sh)
    # midpoints of consecutive collocation points lie on the boundary to second order on panels;
    # keep those well away from every corner (the singular region is resolved only near its nodes)
    mid = 0.5 * (sh.colloc[:-1] + sh.colloc[1:])
    if sh.name == "teardrop":
        corners = np.array([sh.meta["corner"]])
    else:
        corners = sh.meta["vertices"]
    dist = np.min(np.linalg.norm(mid[:, None, :] - corners[None, :, :], axis=2), axis=1)
    seg = np.linalg.norm(sh.colloc[1:] - sh.colloc[:-1], axis=1)
    keep = (dist > 0.05) & (seg < 0.05)
    # exact boundary points: project the midpoints back with the chord error O(seg^2 curvature),
    # which is zero on straight edges; for the teardrop compare against a fine boundary instead
    if sh.name == "cshape":
        pts = mid[keep]
    else:
        fine = w.teardrop2d(levels=12, base_panels=64, q=16, d_frac=0.5).colloc
        dd = np.linalg.norm(fine[:, None, :] - corners[None, :, :], axis=2).min(axis=1)
        pts = fine[dd > 0.05]
    u = phi_matrix(pts, sh.src, KAPPA) @ q
    total = u + np.exp(1j * KAPPA * pts @ D0)
    # measured: teardrop median 1.5e-9, max 5.3e-8; C-shape median 8.7e-9, max 3.7e-7
    assert np.median(np.abs(total)) < 1e-7
    assert np.abs(total).max() < 3e-6


@pytest.mark.parametrize("mode", ["given", "paper"])
def test_scattering_matrix_of_a_cshape_reproduces_its_mfs_solution(mode):
    """S v_hat radiates (through the equivalent points) the field of the plain MFS solution."""
    sh = w.cshape2d(levels=6, base_per_edge=3, d_frac=0.5)
    u_ref, _ = _mfs_far_field(sh)
    if mode == "given":
        # the ring of equivalent points (radius 0.70) passes close to the corners (radius 0.65),
        # which costs accuracy: measured 1e-7
        S = local_s.s_given_points(sh, KAPPA)
        xh = sh.eqpts
        tol = 1e-6
    else:
        S, I_hat = local_s.s_paper_mode(sh, KAPPA, eps_skel=1e-12)
        xh = sh.colloc[I_hat]
        tol = 1e-8
    qhat = S @ (-np.exp(1j * KAPPA * xh @ D0))
    u = gs.field(xh, KAPPA, qhat, FAR)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < tol


# ------------------------------------------------------------------------------------------ rod ---
# A rod (Sec. 5.1 Example 4): a thin rectangle with semicircular caps.  No corners, but the
# curvature jumps where the caps meet the sides; the panels are refined toward those junctions.

def test_rod_far_field_converges_with_junction_refinement():
    fields = [_mfs_far_field(w.rod2d(levels=L))[0] for L in (2, 4, 6)]
    d1 = np.abs(fields[0] - fields[2]).max() / np.abs(fields[2]).max()
    d2 = np.abs(fields[1] - fields[2]).max() / np.abs(fields[2]).max()
    assert d2 < 0.3 * d1
    assert d2 < 1e-8              # measured 1.2e-10 (d1 6.4e-9)


def test_rod_boundary_condition_on_exact_boundary_points():
    """The sound-soft condition on 1600 exact boundary points of the four pieces (straight sides and
    caps, parametrised exactly), away from the four junctions."""
    from workloads.shapes import _rod_pieces

    sh = w.rod2d()
    _, q = _mfs_far_field(sh)
    pts = np.concatenate([piece(np.linspace(0.0, 1.0, 401))[0]
                          for piece, _ in _rod_pieces(sh.meta["half_length"], sh.meta["radius"])])
    d = np.min(np.linalg.norm(pts[:, None, :] - sh.meta["junctions"][None, :, :], axis=2), axis=1)
    pts = pts[d > 0.02]
    total = phi_matrix(pts, sh.src, KAPPA) @ q + np.exp(1j * KAPPA * pts @ D0)
    # measured: median 3.4e-9, max 1.6e-7
    assert np.median(np.abs(total)) < 1e-7
    assert np.abs(total).max() < 2e-6


@pytest.mark.parametrize("mode", ["given", "paper"])
def test_scattering_matrix_of_a_rod_reproduces_its_mfs_solution(mode):
    sh = w.rod2d()
    u_ref, _ = _mfs_far_field(sh)
    if mode == "given":
        S = local_s.s_given_points(sh, KAPPA)
        xh, tol = sh.eqpts, 1e-6   # measured 1.1e-7
    else:
        S, I_hat = local_s.s_paper_mode(sh, KAPPA, eps_skel=1e-12)
        xh, tol = sh.colloc[I_hat], 1e-8   # measured 1.8e-9
    qhat = S @ (-np.exp(1j * KAPPA * xh @ D0))
    u = gs.field(xh, KAPPA, qhat, FAR)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < tol
