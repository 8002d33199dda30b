"""The symmetric pair kernel on the GPU against the FP64 oracle.

With 1 to 32 right-hand sides in FP32 and every body holding a multiple of 64 points, the operator
evaluates phi once per unordered pair and adds it into both sums (G_hat is symmetric).  Its
schedule (groups of 256 points meeting at cyclic distances, one-sided at distance 0 and G/2) has
edge cases in the number of groups G: 1, 2 (both one-sided), odd and even G, a last group with
fewer than four tiles, and every way of cutting the distances into chunks; every test runs with one
wave per block and with eight waves sharing each source tile.  Each case is held to
the oracle at the FP32 budget, and near body pairs exercise the Hankel branches below z = 100.
"""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, crandn, entrywise_err, make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(params=["one_wave", "shared"])
def mfs(gpu_lib, request):
    """Both forms of the kernel: one wave per block (the default where the slices fit the budget),
    and eight waves sharing each source tile (forced by a one-byte slice budget)."""
    gpu_lib.tune_clear()
    gpu_lib.sym_slice_budget(1 if request.param == "shared" else 0)
    yield gpu_lib
    gpu_lib.sym_slice_budget(0)
    gpu_lib.tune_clear()


def _torch():
    import torch

    return torch


def _scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


def _ghat32(mfs, gsc, q):
    torch = _torch()
    t = torch.empty(q.shape, dtype=torch.complex64, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), t, mfs.MFS_FP32)
    return t.cpu().numpy()


def _disks(T):
    """T disks of 64 equivalent points, the first T of a 4 x 4 grid of spacing 3 (kappa 5): near
    body pairs, where the kernel takes the Hankel branches below z = 100."""
    base = w.c1_disks16(T=16)
    return w.Scene(dim=2, kappa=base.kappa, shapes=base.shapes, shape_of=np.zeros(T, np.int32),
                   centres=base.centres[:T].copy(), directions=base.directions, name=f"disks{T}")


def _starfish(T):
    """T starfish (128 points) from the 2000-body scene, far apart (kappa 10)."""
    return w.make_scene("starfish2000", T=T)


def _spheres64(T):
    sh = w.sphere3d(m=300, n=150, k=192, p=300)
    centres = w.random_centres(T, 3, 9.0, 3.2, 4)
    return w.Scene(dim=3, kappa=2.0, shapes=[sh], shape_of=np.zeros(T, np.int32), centres=centres,
                   directions=np.array([[0.0, 0.0, 1.0]]), name="spheres192")


CASES = [("disks", 1), ("disks", 3), ("disks", 4), ("disks", 5), ("disks", 8), ("disks", 9), ("disks", 13),
         ("disks", 16), ("starfish", 2), ("starfish", 3), ("starfish", 7), ("starfish", 40),
         ("spheres", 6)]


@pytest.mark.parametrize("kind,T", CASES)
def test_symmetric_kernel_matches_oracle(mfs, kind, T):
    sc = {"disks": _disks, "starfish": _starfish, "spheres": _spheres64}[kind](T)
    print(f"symmetric ghat {kind} T={T}", flush=True)
    gsc, _ = _scene(mfs, sc)
    assert mfs.tune_get(gsc, 1, mfs.MFS_FP32)["symmetric"] == 1  # the heuristic's choice here
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(31), 1, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    budget = FP32_OPERATOR_TOL
    sym = _ghat32(mfs, gsc, q)
    assert entrywise_err(sym, ref) < budget
    # the plain kernel on the same scene, for comparison
    mfs.tune_set(gsc, 1, mfs.MFS_FP32, 4, 1, 0)
    assert mfs.tune_get(gsc, 1, mfs.MFS_FP32)["symmetric"] == 0
    plain = _ghat32(mfs, gsc, q)
    assert entrywise_err(plain, ref) < budget
    # every way of cutting the group distances into chunks gives the same operator
    for nch in (1, 2, 3, 1024):
        mfs.tune_set(gsc, 1, mfs.MFS_FP32, nch, 0, 1)
        assert mfs.tune_get(gsc, 1, mfs.MFS_FP32)["symmetric"] == 1
        assert entrywise_err(_ghat32(mfs, gsc, q), ref) < budget
    gsc.close()


def test_symmetric_kernel_is_deterministic_and_used_only_where_it_applies(mfs):
    torch = _torch()
    sc = _starfish(24)
    gsc, Ss = _scene(mfs, sc)
    mfs.tune_set(gsc, 1, mfs.MFS_FP32, 8, 0, 1)
    assert mfs.tune_get(gsc, 1, mfs.MFS_FP32)["symmetric"] == 1
    q = crandn(np.random.default_rng(32), 1, gsc.N)
    a, b = _ghat32(mfs, gsc, q), _ghat32(mfs, gsc, q)
    assert np.array_equal(a, b)
    # more than 32 right-hand sides (matrix cores), FP64, or bodies that would need too much
    # padding to whole 64-point tiles (37 points -> 64): other kernels
    for R, prec in ((33, mfs.MFS_FP32), (1, mfs.MFS_FP64)):
        mfs.tune_set(gsc, R, prec, 8, 0, 1)
        assert mfs.tune_get(gsc, R, prec)["symmetric"] == 0
    sh = w.disk2d(radius=0.5, m=80, n=40, src_radius=0.35, k=37, rho_eq=0.6, p=81, r_psi=0.7)
    odd = w.Scene(dim=2, kappa=7.0, shapes=[sh], shape_of=np.zeros(4, np.int32),
                  centres=w.random_centres(4, 2, 6.0, 1.6, 3), directions=w.plane_wave_directions_2d([0.3]),
                  name="disks37")
    other, _ = _scene(mfs, odd)
    mfs.tune_set(other, 1, mfs.MFS_FP32, 8, 0, 1)
    assert mfs.tune_get(other, 1, mfs.MFS_FP32)["symmetric"] == 0
    other.close()
    # the whole operator (S product reads the ~N/512 extra slices) against the oracle
    xh, ptr, bo = gs.pack(sc)
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    y = torch.empty((1, gsc.N), dtype=torch.complex64, device="cuda")
    mfs.apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), y, mfs.MFS_FP32)
    assert entrywise_err(y.cpu().numpy(), ref) < FP32_OPERATOR_TOL
    gsc.close()


def test_autotune_considers_both_kernels(mfs):
    sc = _starfish(64)
    gsc, _ = _scene(mfs, sc)
    res = mfs.autotune(gsc, R=1, prec=mfs.MFS_MIXED, reps=2)
    assert res["ms_plain"] > 0 and res["n_tried"] >= 6
    got = mfs.tune_get(gsc, 1, mfs.MFS_MIXED)
    assert got["symmetric"] == res["symmetric"] and got["source"] == "scene"
    print("autotune starfish64:", res, flush=True)
    gsc.close()


@pytest.mark.parametrize("kind,T,R", [("disks", 13, 2), ("disks", 9, 3), ("starfish", 40, 5), ("spheres", 6, 3),
                                      ("starfish", 7, 7), ("disks", 16, 13), ("starfish", 24, 32)])
def test_symmetric_kernel_many_rhs(mfs, kind, T, R):
    """2 to 32 right-hand sides: 1, 2 or 4 per thread, ragged last group of right-hand sides."""
    sc = {"disks": _disks, "starfish": _starfish, "spheres": _spheres64}[kind](T)
    print(f"symmetric ghat {kind} T={T} R={R}", flush=True)
    gsc, _ = _scene(mfs, sc)
    # untuned: symmetric up to 24 right-hand sides, the matrix cores above, and from 8 where the
    # matrix cores take split FP16 products
    untuned = mfs.tune_get(gsc, R, mfs.MFS_FP32)["symmetric"]
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 4, 0, 0)
    split16 = mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F16X3
    assert untuned == (1 if R <= 24 and not split16 else 0)
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(33), R, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    budget = FP32_OPERATOR_TOL
    for rt in (1, 2, 4):
        for nch in (1, 3):
            mfs.tune_set(gsc, R, mfs.MFS_FP32, nch, rt, 1)
            got = mfs.tune_get(gsc, R, mfs.MFS_FP32)
            assert got["symmetric"] == 1 and got["rhs_per_thread"] == rt
            t = _ghat32(mfs, gsc, q)
            for r in range(R):
                assert entrywise_err(t[r], ref[r]) < budget, (rt, nch, r)
    gsc.close()


def _ellipses112(T):
    """T ellipses of 112 equivalent points: padded to 128 (two tiles) for the symmetric kernel."""
    sh = w.ellipse2d(m=224, n=112, k=112, p=225)
    centres = w.random_centres(T, 2, 9.0, 1.6, 12)
    return w.Scene(dim=2, kappa=8.0, shapes=[sh], shape_of=np.zeros(T, np.int32), centres=centres,
                   directions=w.plane_wave_directions_2d([0.5, 1.5, 2.5]), name="ellipses112")


@pytest.mark.parametrize("kind,T,R", [("spheres400", 5, 1), ("spheres400", 3, 3), ("ellipses112", 9, 1),
                                      ("ellipses112", 11, 2)])
def test_symmetric_kernel_on_padded_bodies(mfs, kind, T, R):
    """Bodies whose point count is not a multiple of 64: in 2D (ellipses of 112) they are padded to
    whole tiles with zero-charge points at the body centre, and the pair sum, the reduction and the S
    product read the padded rows; in 3D (spheres of 400) the kernel works on 16-point sub-blocks of
    the packed layout instead (no padding).  Both against the oracle and the plain kernel."""
    torch = _torch()
    sc = w.make_scene("spheres1000", T=T) if kind == "spheres400" else _ellipses112(T)
    print(f"padded symmetric {kind} T={T} R={R}", flush=True)
    gsc, Ss = _scene(mfs, sc)
    assert mfs.tune_get(gsc, R, mfs.MFS_FP32)["symmetric"] == 1
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(34), R, xh.shape[0])
    budget = FP32_OPERATOR_TOL
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    for nch in (1, 2):
        mfs.tune_set(gsc, R, mfs.MFS_FP32, nch, 0, 1)
        t = _ghat32(mfs, gsc, q)
        for r in range(R):
            assert entrywise_err(t[r], ref[r]) < budget
    # the whole operator: the S product reads the pair sums from the padded rows
    ref_y = gs.matvec(sc, Ss, xh, ptr, bo, q)
    y = torch.empty((R, gsc.N), dtype=torch.complex64, device="cuda")
    mfs.apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), y, mfs.MFS_FP32)
    yy = y.cpu().numpy()
    for r in range(R):
        assert entrywise_err(yy[r], ref_y[r]) < budget
    # and against the plain kernel on the packed layout
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 4, 0, 0)
    assert mfs.tune_get(gsc, R, mfs.MFS_FP32)["symmetric"] == 0
    plain = _ghat32(mfs, gsc, q)
    assert entrywise_err(plain, t) < 2 * budget
    gsc.close()


def _spheres_k(T, k, seed=9):
    """T small spheres (radius 0.5) of k equivalent points in 3D, centres at least 1.7 apart, kappa 4:
    with k = 48, 80 or 400 the 64-point tiles straddle bodies (16-point sub-blocks)."""
    sh = w.sphere3d(radius=0.5, m=2 * k + 40, n=k, src_radius=0.35, k=k, rho_eq=0.6, p=2 * k + 40, r_psi=0.75)
    centres = w.random_centres(T, 3, 2.2 * T ** (1.0 / 3.0) + 2.0, 1.7, seed)
    return w.Scene(dim=3, kappa=4.0, shapes=[sh], shape_of=np.zeros(T, np.int32), centres=centres,
                   directions=np.array([[1.0, 0.0, 0.0], [0.0, 0.6, 0.8], [0.0, 0.0, 1.0], [0.6, 0.8, 0.0],
                                        [0.0, 1.0, 0.0]]), name=f"spheres{T}_k{k}")


def _two_sphere_shapes(T):
    """3D scene mixing 400- and 48-point spheres: sub-blocks of both kinds in one tile."""
    a = w.sphere3d(radius=0.5, m=440, n=200, src_radius=0.35, k=400, rho_eq=0.6, p=440, r_psi=0.75)
    b = w.sphere3d(radius=0.5, m=140, n=48, src_radius=0.35, k=48, rho_eq=0.6, p=140, r_psi=0.75)
    centres = w.random_centres(T, 3, 2.2 * T ** (1.0 / 3.0) + 2.0, 1.7, 17)
    shape_of = (np.arange(T) % 3 == 0).astype(np.int32)
    return w.Scene(dim=3, kappa=4.0, shapes=[a, b], shape_of=shape_of, centres=centres,
                   directions=np.array([[1.0, 0.0, 0.0], [0.0, 0.6, 0.8], [0.0, 0.0, 1.0]]), name=f"spheres2shape{T}")


@pytest.mark.parametrize("case,T,R", [("k400", 3, 1), ("k400", 7, 2), ("k48", 9, 1), ("k48", 23, 3),
                                      ("k80", 5, 5), ("k400", 1, 1), ("mix", 10, 1), ("mix", 13, 3),
                                      ("k48", 40, 2)])
def test_symmetric_kernel_on_sub_blocks_3d(mfs, case, T, R):
    """3D bodies of 16 n points (not whole 64-point tiles): the symmetric kernel runs on 16-point
    sub-blocks with no padded layout.  Cases: tiles straddling two bodies (400), several bodies in
    one tile (48, 80), a last tile only partly filled (N not a multiple of 64), one body (no pairs),
    two shapes, 1 to 5 right-hand sides with 1, 2 and 4 per thread, 1 to 3 distance chunks; against
    the oracle entry by entry, through G_hat and through the whole operator."""
    torch = _torch()
    sc = _two_sphere_shapes(T) if case == "mix" else _spheres_k(T, int(case[1:]))
    sc.directions = sc.directions[:R]
    print(f"sub-block symmetric {case} T={T} N={sc.N} R={R}", flush=True)
    gsc, Ss = _scene(mfs, sc)
    assert mfs.tune_get(gsc, R, mfs.MFS_FP32)["symmetric"] == 1
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(35), R, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    for rt in ((1, 2, 4) if R > 1 else (1,)):
        for nch in (1, 2, 3):
            mfs.tune_set(gsc, R, mfs.MFS_FP32, nch, rt, 1)
            t = _ghat32(mfs, gsc, q)
            if T == 1:
                assert np.count_nonzero(t) == 0
            else:
                assert entrywise_err(t, ref) < FP32_OPERATOR_TOL, (rt, nch)
    ref_y = gs.matvec(sc, Ss, xh, ptr, bo, q)
    y = torch.empty((R, gsc.N), dtype=torch.complex64, device="cuda")
    mfs.apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), y, mfs.MFS_FP32)
    assert entrywise_err(y.cpu().numpy(), ref_y) < FP32_OPERATOR_TOL
    gsc.close()
