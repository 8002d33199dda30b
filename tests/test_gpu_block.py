"""Block GMRES (one Krylov space for all R right-hand sides, Sec. 2.3 GMRES on eq. mbody2) on the GPU,
against the oracle's dense LU solution of the same system (the solution of (I + S G_hat) q = S v is
unique, so every column must match it to the solve's tolerance) and the oracle's own residual.

Cases: the mixed-precision block solve with a complex64 basis (16 and 64 right-hand sides, the
many-right-hand-side pair kernel on the matrix cores), with the correction cycles deflated by the
first cycle's block space (GCRO), the FP64 block solve with restarts, right-hand
sides that repeat (an exactly rank-deficient block: CholeskyQR marks the dependent columns and the
basis is completed with orthogonalised random vectors), a zero right-hand side (zero solution), and
the block solve against the per-column solve on the same scene (same solutions, far fewer steps)."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import make_gpu_scene, rel_err, s_to_device

pytestmark = pytest.mark.gpu


def _scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


def _check(sc, Ss, q, tol_res, tol_lu, vhat=None):
    xh, ptr, bo = gs.pack(sc)
    vh = gs.plane_wave_vhat(sc, xh) if vhat is None else vhat
    b = gs.rhs(sc, Ss, ptr, vh)
    r = b - gs.matvec(sc, Ss, xh, ptr, bo, q)
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, b)
    for c in range(q.shape[0]):
        nb = np.linalg.norm(b[c])
        if nb == 0.0:
            assert np.abs(q[c]).max() == 0.0
            continue
        assert np.linalg.norm(r[c]) / nb < tol_res, (c, np.linalg.norm(r[c]) / nb)
        assert rel_err(q[c], ref[c]) < tol_lu, (c, rel_err(q[c], ref[c]))


@pytest.mark.parametrize("R", [16, 64])
def test_block_mixed_solve_matches_dense_lu(gpu_lib, R):
    import torch

    mfs = gpu_lib
    sc = w.make_scene("mixed2000_R64", T=24)
    sc.directions = sc.directions[:: 64 // R][:R]
    print(f"block mixed solve: {sc.name} N={sc.N} R={R}", flush=True)
    gsc, Ss = _scene(mfs, sc)
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, restart=300, maxit=20000, max_refine=10, inner_tol=3e-6,
                     prec=mfs.MFS_MIXED, basis32=True, block=True, verbose=1)
    print(f"  {info}", flush=True)
    assert info["relres_max"] <= 1e-8 and info["n_refine"] >= 2
    _check(sc, Ss, q.cpu().numpy(), 2e-8, 1e-6)
    # the per-column solve on the same scene: same answer, many more operator applications
    q1 = torch.empty_like(v)
    info1 = mfs.solve(gsc, v, q1, tol=1e-8, restart=600, maxit=20000, max_refine=10, inner_tol=3e-6,
                      prec=mfs.MFS_MIXED, basis32=True)
    print(f"  per column: {info1}", flush=True)
    assert info["n_matvec32"] < info1["n_matvec32"]
    for c in range(R):
        assert rel_err(q.cpu().numpy()[c], q1.cpu().numpy()[c]) < 1e-6
    gsc.close()


def test_block_fp64_solve_with_restarts(gpu_lib):
    import torch

    mfs = gpu_lib
    sc = w.make_scene("disks16")
    sc.directions = w.plane_wave_directions_2d(np.linspace(0.0, 5.5, 8))
    gsc, Ss = _scene(mfs, sc)
    v = torch.empty((8, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-10, restart=4, maxit=2000, prec=mfs.MFS_FP64, block=True, verbose=1)
    print(f"  {info}", flush=True)
    assert info["relres_max"] <= 1e-10 and info["n_restart"] > 1 and info["n_matvec32"] == 0
    _check(sc, Ss, q.cpu().numpy(), 2e-10, 1e-8)
    gsc.close()


def test_block_solve_with_repeated_and_zero_right_hand_sides(gpu_lib):
    """Directions a, a, b, c, c, c and one zero data vector: the starting block has rank 3 (plus the
    zero column).  Repeated columns must get identical solutions, the zero column a zero one."""
    import torch

    mfs = gpu_lib
    sc = w.make_scene("starfish2000", T=20)
    ang = [0.3, 0.3, 1.7, 4.0, 4.0, 4.0, 2.2]
    sc.directions = w.plane_wave_directions_2d(ang)
    R = len(ang)
    gsc, Ss = _scene(mfs, sc)
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    v[R - 1].zero_()
    for prec in (mfs.MFS_MIXED, mfs.MFS_FP64):
        q = torch.empty_like(v)
        info = mfs.solve(gsc, v, q, tol=1e-8, restart=200, maxit=5000, max_refine=10, inner_tol=3e-6, prec=prec,
                         basis32=prec == mfs.MFS_MIXED, block=True, verbose=1)
        print(f"  prec {prec}: {info}", flush=True)
        assert info["relres_max"] <= 1e-8
        qh = q.cpu().numpy()
        assert rel_err(qh[1], qh[0]) < 1e-9 and rel_err(qh[4], qh[3]) < 1e-9 and rel_err(qh[5], qh[3]) < 1e-9
        vh = v.cpu().numpy()
        _check(sc, Ss, qh, 2e-8, 1e-6, vhat=vh)
    gsc.close()


def test_block_solve_rejects_what_it_does_not_take(gpu_lib):
    import torch

    mfs = gpu_lib
    sc = w.make_scene("starfish2000", T=4)
    sc.directions = w.plane_wave_directions_2d(np.linspace(0.0, 3.0, 65))
    gsc, _ = _scene(mfs, sc)
    v = torch.zeros((65, gsc.N), dtype=torch.complex128, device="cuda")
    with pytest.raises(mfs.MfsError):
        mfs.solve(gsc, v, torch.empty_like(v), prec=mfs.MFS_MIXED, block=True)  # more than 64 columns
    v2 = v[:2].contiguous()
    with pytest.raises(mfs.MfsError):
        mfs.solve(gsc, v2, torch.empty_like(v2), prec=mfs.MFS_MIXED, block=True, use_graph=True)
    gsc.close()


@pytest.mark.parametrize("key,T,R", [("mixed2000_R64", 60, 64), ("starfish2000", 40, 8)])
def test_block_deflated_correction_cycles(gpu_lib, key, T, R):
    """deflate with block: the correction cycles run on (I - C C^H) K~ with C from the first cycle's
    kept block space; same solution as the dense LU, fewer block steps in the corrections than the
    plain restart, and the same first cycle."""
    import torch

    mfs = gpu_lib
    sc = w.make_scene(key, T=T)
    sc.directions = w.plane_wave_directions_2d(2.0 * np.pi * np.arange(R) / R)
    print(f"deflated block solve: {sc.name} N={sc.N} R={R}", flush=True)
    gsc, Ss = _scene(mfs, sc)
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    runs = {}
    for deflate in (False, True):
        q = torch.empty_like(v)
        info = mfs.solve(gsc, v, q, tol=1e-8, restart=400, maxit=20000, max_refine=10, inner_tol=3e-6,
                         prec=mfs.MFS_MIXED, basis32=True, block=True, deflate=deflate, verbose=1)
        print(f"  deflate={deflate}: {info}", flush=True)
        assert info["relres_max"] <= 1e-8
        runs[deflate] = (q.cpu().numpy(), info)
    _check(sc, Ss, runs[True][0], 2e-8, 1e-6)
    assert runs[True][1]["n_matvec32"] < runs[False][1]["n_matvec32"]
    for c in range(R):
        assert rel_err(runs[True][0][c], runs[False][0][c]) < 1e-6
    gsc.close()
