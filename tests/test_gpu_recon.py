"""Parity of the GPU reconstruction of full MFS sources and of the near-body field (Sec. 4.6) with
the FP64 oracle, through the C ABI.

The oracle and the GPU get the same equivalent sources (the oracle's dense solve), so these tests
isolate the reconstruction and the near-field evaluation.  The least-squares pseudo-inverse differs
between the two (truncated SVD against pivoted QR), so parity is on the field the sources produce
near and on the bodies, which is unique; both are also held to the physics (series, multipole
solution, boundary condition).
"""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s, reconstruct as rc
from tests.analytic import MultiDisk, disk_series
from tests.gpu_helpers import make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _near_points(centre, radii, count, phase=0.13):
    return np.concatenate([centre[None, :] + w.circle_points(count, r, phase + 0.37 * i)
                           for i, r in enumerate(radii)], 0)


def _setup(mfs, sc):
    """Oracle solve of the scene, the GPU scene with the oracle's S, and reconstruction factors."""
    torch = _torch()
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    xh, ptr, bo = gs.pack(sc)
    q = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    recons = [mfs.Recon(s, sc.kappa) for s in sc.shapes]
    R = q.shape[0]
    mt, nt = mfs.near_sizes(gsc, recons)
    v = torch.empty((R, mt), dtype=torch.complex128, device="cuda")
    mfs.plane_wave_colloc(gsc, recons, sc.directions[:R], v)
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    qm = torch.empty((R, nt), dtype=torch.complex128, device="cuda")
    mfs.reconstruct(gsc, recons, v, qd, qm)
    torch.cuda.synchronize()
    return dict(gsc=gsc, recons=recons, q=q, qd=qd, qm=qm, v=v, xh=xh, bo=bo, Ss=Ss)


def _gpu_field(mfs, st, targets):
    torch = _torch()
    tg = torch.from_numpy(np.ascontiguousarray(targets)).cuda()
    u = torch.empty((st["q"].shape[0], targets.shape[0]), dtype=torch.complex128, device="cuda")
    mfs.eval_field_near(st["gsc"], st["recons"], st["qd"], st["qm"], tg, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _oracle_near(sc, st):
    U = [rc.incoming_map(s, sc.kappa) for s in sc.shapes]
    return rc.reconstruct_mfs(sc, U, st["xh"], st["bo"], st["q"], rc.plane_wave_on_boundary(sc, sc.directions),
                              workers=4)


def test_plane_wave_on_boundary_matches_oracle(gpu_lib):
    sc = w.make_scene("mixed2000_R64", T=7)
    sc.directions = sc.directions[:3]
    st = _setup(gpu_lib, sc)
    ref = rc.plane_wave_on_boundary(sc, sc.directions)
    assert np.abs(st["v"].cpu().numpy() - ref).max() < 1e-13


def test_single_disk_near_field_matches_series(gpu_lib):
    sc = w.c1_disks16(T=1)
    st = _setup(gpu_lib, sc)
    tg = _near_points(sc.centres[0], [1.0, 1.02, 1.2, 1.45, 1.6, 2.5], 41)
    u = _gpu_field(gpu_lib, st, tg)[0]
    ref = disk_series(sc.kappa, 1.0, 0.0, tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-8  # the oracle measures 3.2e-9


def test_sixteen_disks_near_field_matches_oracle_and_multipole(gpu_lib):
    sc = w.c1_disks16()
    st = _setup(gpu_lib, sc)
    tg = np.concatenate([_near_points(sc.centres[t], [1.0, 1.1, 1.3, 1.49, 1.7], 23, 0.05 * t)
                         for t in (0, 5, 10, 15)])
    u = _gpu_field(gpu_lib, st, tg)[0]
    u_ref = rc.field_near(sc, st["xh"], st["q"], _oracle_near(sc, st), tg)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-10
    mp = MultiDisk(sc.kappa, 1.0, sc.centres, 0.0, nmax=25).field(tg)
    assert np.abs(u - mp).max() / np.abs(mp).max() < 1e-7


def _fine_starfish(T):
    base = w.make_scene("starfish2000", T=T)
    sh = w.starfish2d(m=512, n=256, p=513)
    return w.Scene(dim=2, kappa=base.kappa, shapes=[sh], shape_of=base.shape_of, centres=base.centres,
                   directions=base.directions, name=f"starfish{T}_fine")


def test_starfish_boundary_condition_and_oracle_parity(gpu_lib):
    sc = _fine_starfish(6)
    st = _setup(gpu_lib, sc)
    chk = w.starfish2d(m=2048, n=16).colloc
    pts = np.concatenate([chk + sc.centres[t][None, :] for t in range(sc.T)])
    u = _gpu_field(gpu_lib, st, pts)[0]
    total = u + np.exp(1j * sc.kappa * pts @ sc.directions[0])
    assert np.abs(total).max() < 1e-6  # the oracle measures 1.4e-7
    u_ref = rc.field_near(sc, st["xh"], st["q"], _oracle_near(sc, st), pts)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-9


def _ragged_scene():
    a = w.disk2d(radius=0.5, m=80, n=40, src_radius=0.35, k=37, rho_eq=0.6, p=81, r_psi=0.7)
    b = w.ellipse2d(a=0.6, b=0.3, m=140, n=70, d=0.05, k=70, rho_eq=0.65, p=141, r_psi=0.72)
    centres = w.random_centres(9, 2, 8.0, 1.6, 77)
    return w.Scene(dim=2, kappa=7.0, shapes=[a, b], shape_of=np.array([0, 1, 1, 0, 1, 0, 0, 1, 1], np.int32),
                   centres=centres, directions=w.plane_wave_directions_2d([0.3, 2.2]), name="ragged")


def test_two_shapes_two_directions_match_oracle(gpu_lib):
    sc = _ragged_scene()
    st = _setup(gpu_lib, sc)
    tg = np.concatenate([_near_points(sc.centres[t], [0.55, 0.68, 0.9], 17, 0.1 * t) for t in range(sc.T)])
    u = _gpu_field(gpu_lib, st, tg)
    u_ref = rc.field_near(sc, st["xh"], st["q"], _oracle_near(sc, st), tg)
    for r in range(2):
        assert np.abs(u[r] - u_ref[r]).max() / np.abs(u_ref[r]).max() < 1e-9


def test_spheres_near_field_matches_oracle(gpu_lib):
    sc = w.make_scene("spheres1000", T=4)
    st = _setup(gpu_lib, sc)
    rng = np.random.default_rng(3)
    dirs = rng.normal(size=(60, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    tg = np.concatenate([sc.centres[t][None, :] + dirs * r for t in (0, 2) for r in (1.05, 1.3, 1.45)])
    u = _gpu_field(gpu_lib, st, tg)[0]
    u_ref = rc.field_near(sc, st["xh"], st["q"], _oracle_near(sc, st), tg)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-9


def test_reconstructed_sources_match_oracle_where_full_rank(gpu_lib):
    """Where A has full numerical rank its least-squares solution is unique, so the sources agree."""
    sc = w.c1_disks16(T=4)
    st = _setup(gpu_lib, sc)
    assert st["recons"][0].rank == sc.shapes[0].src.shape[0]
    ref = _oracle_near(sc, st)
    got = st["qm"].cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-8


def test_invalid_reconstruction_arguments(gpu_lib):
    mfs = gpu_lib
    sc = w.c1_disks16(T=4)
    st = _setup(mfs, sc)
    other = mfs.Recon(sc.shapes[0], sc.kappa * 2.0)  # wrong wavenumber for this scene
    with pytest.raises(mfs.MfsError):
        mfs.near_sizes(st["gsc"], [other])
    other.close()


def test_replaced_factors_are_picked_up(gpu_lib):
    """A scene caches its near-field tables per set of factors; new factors (even at a reused
    address) must replace them: the field with the second set equals a fresh scene's."""
    mfs = gpu_lib
    torch = _torch()
    sc = w.c1_disks16(T=4)
    st = _setup(mfs, sc)
    tg = np.concatenate([_near_points(sc.centres[t], [1.1, 1.4], 11) for t in range(sc.T)])
    first = _gpu_field(mfs, st, tg)
    for r in st["recons"]:
        r.close()
    # smaller proxy radius: targets at 1.4 now use the equivalent points instead of the MFS sources
    st["recons"] = [mfs.Recon(s, sc.kappa, psi_radius=1.3) for s in sc.shapes]
    second = _gpu_field(mfs, st, tg)
    fresh = _setup(mfs, sc)
    fresh["recons"] = [mfs.Recon(s, sc.kappa, psi_radius=1.3) for s in sc.shapes]
    ref = _gpu_field(mfs, fresh, tg)
    assert np.array_equal(second, ref)
    # and the new radius did take effect (targets at 1.4 switched representation)
    assert not np.array_equal(first, second)
