"""Bodies with corners on the GPU: scattering matrices built by mfs_build_S for panel-discretised
shapes with dyadic corner refinement, and a scene mixing smooth and cornered bodies solved through
the C ABI.  References: the plain MFS solution of each shape (oracle), the oracle's dense solve, and
the sound-soft boundary condition on every body."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s, reconstruct as rc
from oracle.fundamental import phi_matrix

pytestmark = pytest.mark.gpu

KAPPA = 10.0
D0 = np.array([np.cos(0.3), np.sin(0.3)])
FAR = w.circle_points(48, 3.0, 0.1)


def _torch():
    import torch

    return torch


def _mfs_far(sh):
    A = phi_matrix(sh.colloc, sh.src, KAPPA)
    q = local_s.tsvd_solve(A, -np.exp(1j * KAPPA * sh.colloc @ D0), 1e-13)
    return phi_matrix(FAR, sh.src, KAPPA) @ q


SHAPES = {
    "teardrop": lambda: w.teardrop2d(levels=8, base_panels=16, d_frac=0.5),
    "cshape": lambda: w.cshape2d(levels=6, base_per_edge=3, d_frac=0.5),
    "rod": lambda: w.rod2d(levels=4),
}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("paper", [False, True])
def test_build_S_on_cornered_shape_reproduces_mfs_solution(gpu_lib, name, paper):
    mfs = gpu_lib
    sh = SHAPES[name]()
    u_ref = _mfs_far(sh)
    b = mfs.build_S(sh, KAPPA, paper_mode=paper, eps_skel=1e-12)
    S = b.S64.cpu().numpy().T  # column-major storage -> row-major matrix
    xh = sh.colloc[b.skel_idx] if paper else sh.eqpts
    qhat = S @ (-np.exp(1j * KAPPA * xh @ D0))
    u = gs.field(xh, KAPPA, qhat, FAR)[0]
    err = np.abs(u - u_ref).max() / np.abs(u_ref).max()
    # the oracle measures 1e-7 with the ring of equivalent points (it passes near the C-shape's
    # corners) and 1e-8 or better with the skeleton.  The rod is thin (aspect 6): its MFS matrix is
    # the worst conditioned, and the pivoted-QR basic solution gives 1.9e-8 with the skeleton
    # where the oracle's truncated SVD gives 2.2e-9 (both fit the same data; they differ in the
    # near-null space)
    tol = 1e-6 if not paper else (5e-8 if name == "rod" else 1e-8)
    assert err < tol, err


def _mixed_corner_scene(T=9):
    # the starfish at m = 512: at the workload's m = 256 its own MFS fit leaves 1.5e-4 on its boundary
    shapes = [w.starfish2d(m=512, n=256, p=513), SHAPES["teardrop"](), SHAPES["cshape"]()]
    rng = np.random.default_rng(31)
    centres = w.random_centres(T, 2, 7.0, 1.6, 31)
    shape_of = (np.arange(T) % 3).astype(np.int32)
    rng.shuffle(shape_of)
    return w.Scene(dim=2, kappa=KAPPA, shapes=shapes, shape_of=shape_of, centres=centres,
                   directions=w.plane_wave_directions_2d([0.3]), name="corners9")


def test_scene_with_cornered_bodies_solves_and_meets_boundary_condition(gpu_lib):
    mfs = gpu_lib
    torch = _torch()
    sc = _mixed_corner_scene()
    built = [mfs.build_S(s, KAPPA) for s in sc.shapes]
    scene = mfs.Scene(2, KAPPA, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                      [b.S64 for b in built], [b.S32 for b in built])
    v = torch.empty((1, scene.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(scene, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(scene, v, q, tol=1e-10, restart=300, prec=mfs.MFS_FP64)
    assert info["relres_max"] <= 1e-10
    # against the oracle's dense solve with its own S
    Ss = [local_s.s_given_points(s, KAPPA) for s in sc.shapes]
    xh, ptr, bo = gs.pack(sc)
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    tg = w.far_targets(sc, 64)
    u = gs.field(xh, KAPPA, q.cpu().numpy(), tg)[0]
    u_ref = gs.field(xh, KAPPA, ref, tg)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-8
    # sound-soft condition on every body, between collocation points, through the reconstruction
    recons = [mfs.Recon(s, KAPPA) for s in sc.shapes]
    mt, nt = mfs.near_sizes(scene, recons)
    vc = torch.empty((1, mt), dtype=torch.complex128, device="cuda")
    mfs.plane_wave_colloc(scene, recons, sc.directions, vc)
    qm = torch.empty((1, nt), dtype=torch.complex128, device="cuda")
    mfs.reconstruct(scene, recons, vc, q, qm)
    # boundary points between the collocation points, away from the corners: exact points of a finer
    # discretisation for the curved bodies (chord midpoints would lie off a curved boundary), edge
    # midpoints for the C-shape's straight edges
    fine_td = w.teardrop2d(levels=8, base_panels=64, q=16, d_frac=0.5)
    td_pts = fine_td.colloc[np.linalg.norm(fine_td.colloc - fine_td.meta["corner"][None, :], axis=1) > 0.05]
    worst = {}
    for t in range(sc.T):
        sh = sc.shapes[int(sc.shape_of[t])]
        if sh.name == "teardrop":
            body = td_pts
        elif sh.name == "starfish":
            body = w.starfish2d(m=2048, n=16).colloc
        else:
            mid = 0.5 * (sh.colloc[:-1] + sh.colloc[1:])
            seg = np.linalg.norm(sh.colloc[1:] - sh.colloc[:-1], axis=1)
            body = mid[seg < 0.02]
            d = np.min(np.linalg.norm(body[:, None, :] - sh.meta["vertices"][None, :, :], axis=2), axis=1)
            body = body[d > 0.05]
        pts = body + sc.centres[t][None, :]
        tgd = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        ud = torch.empty((1, pts.shape[0]), dtype=torch.complex128, device="cuda")
        mfs.eval_field_near(scene, recons, q, qm, tgd, ud)
        total = ud.cpu().numpy()[0] + np.exp(1j * KAPPA * pts @ sc.directions[0])
        worst[sh.name] = max(worst.get(sh.name, 0.0), float(np.abs(total).max()))
    # the oracle measures 1.1e-7 (starfish), 4.5e-6 (teardrop), 2.1e-5 (C-shape) on this scene
    assert worst["starfish"] < 1e-6 and worst["teardrop"] < 3e-5 and worst["cshape"] < 1e-4, worst
    for r in recons:
        r.close()
    scene.close()
