"""Rotated copies of a shape on the GPU: packing, solves and the near field for scenes whose bodies
are turned copies sharing one S, against the oracle (which places the same turned point sets)."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s, reconstruct as rc
from tests.gpu_helpers import make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _scene(dim):
    if dim == 2:
        shapes = [w.kite2d(m=512, n=256, d=0.02, k=128, p=257), w.ellipse2d()]
        centres = w.random_centres(6, 2, 6.0, 1.6, 5)
        return w.Scene(dim=2, kappa=6.0, shapes=shapes, shape_of=np.arange(6) % 2, centres=centres,
                       directions=w.plane_wave_directions_2d([0.4, 1.9]), name="rot2",
                       rotations=w.random_rotations(6, 2, 6))
    shapes = [w.ellipsoid3d(m=400, n=200, k=192, p=400), w.torus3d(n_u=40, n_v=20, k=192, p=600)]
    centres = w.random_centres(4, 3, 6.0, 3.2, 7)
    return w.Scene(dim=3, kappa=2.0, shapes=shapes, shape_of=np.arange(4) % 2, centres=centres,
                   directions=np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]]), name="rot3",
                   rotations=w.random_rotations(4, 3, 8))


def _setup(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


@pytest.mark.parametrize("dim", [2, 3])
def test_rotated_packing_matches_oracle(gpu_lib, dim):
    sc = _scene(dim)
    gsc, _ = _setup(gpu_lib, sc)
    xh, _, _ = gs.pack(sc)
    assert np.abs(gsc.points() - xh).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_rotated_scene_solves_match_oracle(gpu_lib, dim):
    mfs = gpu_lib
    torch = _torch()
    sc = _scene(dim)
    gsc, Ss = _setup(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    R = sc.R
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    tg = w.far_targets(sc, 48)
    u_ref = gs.field(xh, sc.kappa, ref, tg)
    for prec, tol in ((mfs.MFS_FP64, 1e-9), (mfs.MFS_MIXED, 1e-6)):
        q = torch.empty_like(v)
        info = mfs.solve(gsc, v, q, tol=1e-10 if prec == mfs.MFS_FP64 else 1e-8, restart=300, prec=prec,
                         basis32=prec == mfs.MFS_MIXED)
        u = gs.field(xh, sc.kappa, q.cpu().numpy(), tg)
        for r in range(R):
            assert np.abs(u[r] - u_ref[r]).max() / np.abs(u_ref[r]).max() < tol, (prec, r, info)


def test_rotated_near_field_matches_oracle(gpu_lib):
    mfs = gpu_lib
    torch = _torch()
    sc = _scene(2)
    gsc, Ss = _setup(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    q = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    recons = [mfs.Recon(s, sc.kappa) for s in sc.shapes]
    mt, nt = mfs.near_sizes(gsc, recons)
    R = sc.R
    vc = torch.empty((R, mt), dtype=torch.complex128, device="cuda")
    mfs.plane_wave_colloc(gsc, recons, sc.directions, vc)
    assert np.abs(vc.cpu().numpy() - rc.plane_wave_on_boundary(sc)).max() < 1e-13
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    qm = torch.empty((R, nt), dtype=torch.complex128, device="cuda")
    mfs.reconstruct(gsc, recons, vc, qd, qm)
    tg = np.concatenate([sc.place(t, 1.05 * sc.shapes[int(sc.shape_of[t])].colloc[::9]) for t in range(sc.T)])
    u = torch.empty((R, tg.shape[0]), dtype=torch.complex128, device="cuda")
    mfs.eval_field_near(gsc, recons, qd, qm, torch.from_numpy(tg).cuda(), u)
    U = [rc.incoming_map(s, sc.kappa) for s in sc.shapes]
    qm_ref = rc.reconstruct_mfs(sc, U, xh, bo, q, rc.plane_wave_on_boundary(sc), workers=4)
    u_ref = rc.field_near(sc, xh, q, qm_ref, tg)
    got = u.cpu().numpy()
    for r in range(R):
        assert np.abs(got[r] - u_ref[r]).max() / np.abs(u_ref[r]).max() < 1e-9
    for rr in recons:
        rr.close()
