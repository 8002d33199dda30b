"""Pins for rotated copies of a shape sharing one scattering matrix, and for the torus.

phi depends only on distances, so a body whose point sets are all turned by Q has the same A, B, D,
B_hat and hence the same S.  The pins: turning a whole configuration (bodies, centres and incident
direction) by Q turns the scattered field by Q, in 2D and 3D, far and near; a torus's S reproduces
its plain MFS solution, and the torus's field converges under grid refinement.
"""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s, reconstruct as rc
from oracle.fundamental import phi_matrix


def _rot2(a):
    return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])


def _solve(sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    xh, ptr, bo = gs.pack(sc)
    q = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    return xh, bo, q


def _turned(sc, Q):
    """The same configuration turned by Q about the origin."""
    R0 = sc.rotations if sc.rotations is not None else np.tile(np.eye(sc.dim), (sc.T, 1, 1))
    return w.Scene(dim=sc.dim, kappa=sc.kappa, shapes=sc.shapes, shape_of=sc.shape_of,
                   centres=sc.centres @ Q.T, directions=sc.directions @ Q.T, name=sc.name + "_turned",
                   rotations=np.einsum("ij,tjk->tik", Q, R0))


@pytest.mark.parametrize("dim", [2, 3])
def test_turning_the_configuration_turns_the_field(dim):
    if dim == 2:
        shapes = [w.kite2d(m=512, n=256, d=0.02, k=128, p=257), w.ellipse2d()]
        centres = w.random_centres(4, 2, 5.0, 1.6, 5)
        rot = w.random_rotations(4, 2, 6)
        Q = _rot2(0.7)
        kappa, dirs = 6.0, w.plane_wave_directions_2d([0.4])
    else:
        shapes = [w.ellipsoid3d(m=400, n=200, k=196, p=400), w.torus3d(n_u=24, n_v=12, k=196, p=400)]
        centres = w.random_centres(3, 3, 6.0, 3.2, 7)
        rot = w.random_rotations(3, 3, 8)
        Q = w.random_rotations(1, 3, 9)[0]
        kappa, dirs = 2.0, np.array([[0.0, 0.6, 0.8]])
    sc = w.Scene(dim=dim, kappa=kappa, shapes=shapes, shape_of=np.arange(centres.shape[0]) % 2,
                 centres=centres, directions=dirs, name="rot", rotations=rot)
    sc2 = _turned(sc, Q)
    xh, bo, q = _solve(sc)
    xh2, bo2, q2 = _solve(sc2)
    # the equivalent points are turned, and the solutions agree entry by entry
    assert np.abs(xh @ Q.T - xh2).max() < 1e-12
    assert np.abs(q - q2).max() / np.abs(q).max() < 1e-9
    tg = w.far_targets(sc, 40)
    u = gs.field(xh, kappa, q, tg)[0]
    u2 = gs.field(xh2, kappa, q2, tg @ Q.T)[0]
    assert np.abs(u - u2).max() / np.abs(u).max() < 1e-10
    # near the first body, through the reconstructed MFS sources
    U = [rc.incoming_map(s, kappa) for s in shapes]
    qm = rc.reconstruct_mfs(sc, U, xh, bo, q, rc.plane_wave_on_boundary(sc), workers=1)
    qm2 = rc.reconstruct_mfs(sc2, U, xh2, bo2, q2, rc.plane_wave_on_boundary(sc2), workers=1)
    near = sc.place(0, 1.02 * shapes[0].colloc[::7])
    a = rc.field_near(sc, xh, q, qm, near)[0]
    b = rc.field_near(sc2, xh2, q2, qm2, near @ Q.T)[0]
    assert np.abs(a - b).max() / np.abs(a).max() < 1e-9


def test_rotated_body_differs_from_unrotated():
    """The pin above is not trivially satisfied: an unsymmetric body's field depends on its turn."""
    sh = w.kite2d(m=512, n=256, d=0.02, k=128, p=257)
    base = dict(dim=2, kappa=6.0, shapes=[sh], shape_of=np.zeros(1, np.int32), centres=np.zeros((1, 2)),
                directions=w.plane_wave_directions_2d([0.4]), name="one")
    sc0 = w.Scene(**base)
    sc1 = w.Scene(**base, rotations=_rot2(0.9)[None])
    tg = w.circle_points(32, 3.0)
    x0, _, q0 = _solve(sc0)
    x1, _, q1 = _solve(sc1)
    u0 = gs.field(x0, 6.0, q0, tg)[0]
    u1 = gs.field(x1, 6.0, q1, tg)[0]
    assert np.abs(u0 - u1).max() / np.abs(u0).max() > 1e-2


def test_torus_scattering_matrix_and_refinement():
    kappa = 2.0
    d = np.array([0.3, 0.4, np.sqrt(1 - 0.25)])
    far = w.fibonacci_sphere(60, 4.0)

    def mfs_far(sh):
        A = phi_matrix(sh.colloc, sh.src, kappa)
        qq = local_s.tsvd_solve(A, -np.exp(1j * kappa * sh.colloc @ d), 1e-13)
        return phi_matrix(far, sh.src, kappa) @ qq

    coarse = w.torus3d(n_u=40, n_v=20, k=256, p=600)
    fine = w.torus3d(n_u=56, n_v=28, k=256, p=600)
    u_c, u_f = mfs_far(coarse), mfs_far(fine)
    assert np.abs(u_c - u_f).max() / np.abs(u_f).max() < 5e-5    # measured 1.2e-5
    S = local_s.s_given_points(coarse, kappa)
    qhat = S @ (-np.exp(1j * kappa * coarse.eqpts @ d))
    u_s = gs.field(coarse.eqpts, kappa, qhat, far)[0]
    assert np.abs(u_s - u_c).max() / np.abs(u_c).max() < 1e-5    # measured 2.3e-6 (256 points on a sphere)
