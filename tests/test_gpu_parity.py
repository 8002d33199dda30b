"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances, per entry of every right-hand side and relative to that right-hand side's largest
reference entry: FP64 kernels 1e-12 (the device Hankel function is accurate to ~2e-15 and sums of N
terms add ~sqrt(N) eps); FP32 pair sums with the body-centre phase split 1e-5 (about 10x their
measured error); FP32 field evaluation on plain single-precision distances its error model
10 (kappa L + 10) 2^-24 (L = scene diameter); S from the
GPU least-squares to 1e-8 relative where the factorisations are full rank (the solution of a
full-rank least-squares problem is unique, so only rounding, amplified by cond ~ 1e4-1e6, differs).
"""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.analytic import disk_series
from tests.gpu_helpers import FP32_OPERATOR_TOL, assert_entrywise, crandn, fp32_distance_budget, make_gpu_scene, \
    rel_err, s_to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfs(gpu_lib):
    return gpu_lib


def _torch():
    import torch

    return torch


def _scene_with_oracle_S(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


def _ragged_scene():
    """Two shapes with k = 37 and 70 (not multiples of the 64-wide wave), 9 bodies."""
    a = w.disk2d(radius=0.5, m=80, n=40, src_radius=0.35, k=37, rho_eq=0.6, p=81, r_psi=0.7)
    b = w.ellipse2d(a=0.6, b=0.3, m=140, n=70, d=0.05, k=70, rho_eq=0.65, p=141, r_psi=0.72)
    centres = w.random_centres(9, 2, 8.0, 1.6, 77)
    return w.Scene(dim=2, kappa=7.0, shapes=[a, b], shape_of=np.array([0, 1, 1, 0, 1, 0, 0, 1, 1], np.int32),
                   centres=centres, directions=w.plane_wave_directions_2d([0.3]), name="ragged")


SMALL_SCENES = {
    "disks16": lambda: w.make_scene("disks16"),
    "starfish32": lambda: w.make_scene("starfish2000", T=32),
    "spheres6": lambda: w.make_scene("spheres1000", T=6),
    "mixed24": lambda: w.make_scene("mixed2000_R64", T=24),
    "ragged9": _ragged_scene,
}


# ------------------------------------------------------------------ build_S ---
@pytest.mark.parametrize("which", ["disk", "starfish", "sphere", "c4disk", "ellipse", "c4star", "kite"])
def test_build_S_given_points_matches_oracle(mfs, which):
    shapes = {"disk": (w.c1_disks16().shapes[0], 5.0), "starfish": (w.c2_starfish2000(T=2).shapes[0], 10.0),
              "sphere": (w.c3_spheres1000(T=1).shapes[0], 3.0), "c4disk": (w.c4_shapes()[0], 20.0),
              "ellipse": (w.c4_shapes()[1], 20.0), "c4star": (w.c4_shapes()[2], 20.0),
              "kite": (w.c4_shapes()[3], 20.0)}
    shape, kappa = shapes[which]
    print(f"build_S given-point mode: {which} m={shape.m} n={shape.n} p={shape.p} k={shape.k}", flush=True)
    built = mfs.build_S(shape, kappa)
    S_gpu = built.matrix64().cpu().numpy()
    S_ref = local_s.s_given_points(shape, kappa)
    assert built.k == shape.k
    if which != "kite":
        # A and B_hat have full numerical rank (cond <= 1e7), so the least-squares solutions are
        # unique and the matrices agree entry by entry up to rounding amplified by the condition
        assert built.diag[0] == shape.n and built.diag[1] == shape.k
        assert rel_err(S_gpu, S_ref) < 1e-8
    # the kite's A has cond ~1e16 (rank deficient at eps_ls): pivoted-QR basic and truncated-SVD
    # minimum-norm solutions differ in the null space, so only the action of S is compared, to
    # the level of the discretisation's own error (both are 2e-8 from a 4x finer MFS solve, and
    # 5e-8 apart, in a float64 model of both factorisations)
    # FP32 copy is the rounded FP64 matrix
    assert rel_err(built.matrix32().cpu().numpy(), S_gpu) < 1e-7
    # action on an incoming plane wave, observed in the far field
    d = np.zeros(shape.eqpts.shape[1])
    d[0] = 1.0
    vhat = -np.exp(1j * kappa * shape.eqpts @ d)
    tg = (w.circle_points(23, 4.0, 0.2) if shape.eqpts.shape[1] == 2 else w.fibonacci_sphere(23, 4.0))
    u_gpu = gs.field(shape.eqpts, kappa, S_gpu @ vhat, tg)
    u_ref = gs.field(shape.eqpts, kappa, S_ref @ vhat, tg)
    assert rel_err(u_gpu, u_ref) < (3e-7 if which == "kite" else 1e-10)


def test_build_S_kite_matches_fine_plain_mfs(mfs):
    """Rank-deficient case pinned to physics: the GPU-built kite S against a 4x finer classical
    MFS least-squares solve of the same single-body problem."""
    from oracle import fundamental

    shape, kappa = w.c4_shapes()[3], 20.0
    S = mfs.build_S(shape, kappa).matrix64().cpu().numpy()
    fine = w.kite2d(bounding=0.65, m=2048, n=1024, d=0.03)
    A = fundamental.phi_matrix(fine.colloc, fine.src, kappa)
    tg = w.circle_points(41, 3.0, 0.2)
    for ang in (0.0, 1.1):
        d = np.array([np.cos(ang), np.sin(ang)])
        qf = np.linalg.lstsq(A, -np.exp(1j * kappa * fine.colloc @ d), rcond=1e-14)[0]
        ref = fundamental.phi_matrix(tg, fine.src, kappa) @ qf
        u = gs.field(shape.eqpts, kappa, S @ (-np.exp(1j * kappa * shape.eqpts @ d)), tg)[0]
        assert np.abs(u - ref).max() / np.abs(ref).max() < 3e-7


def test_build_S_paper_mode_disk_matches_series(mfs):
    shape = w.disk2d(radius=1.0, m=128, n=64, src_radius=0.7, k=64, rho_eq=1.2, p=128, r_psi=1.5)
    built = mfs.build_S(shape, 5.0, paper_mode=True, eps_skel=1e-12)
    _, I_ref = local_s.s_paper_mode(shape, 5.0, eps_skel=1e-12)
    assert abs(built.k - I_ref.size) <= 2
    xh = shape.colloc[built.skel_idx]
    S = built.matrix64().cpu().numpy()
    tg = w.circle_points(29, 2.5, 0.1)
    u = gs.field(xh, 5.0, S @ (-np.exp(5j * xh[:, 0])), tg)[0]
    ref = disk_series(5.0, 1.0, 0.0, tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-9


def test_build_S_paper_mode_starfish_matches_oracle_action(mfs):
    shape = w.starfish2d(m=192, n=96, d=0.1, k=60, rho_eq=0.67, p=193, r_psi=1.5, r0=81 / 101, amp=-20 / 81)
    built = mfs.build_S(shape, 10.0, paper_mode=True, eps_skel=1e-10)
    S_ref, I_ref = local_s.s_paper_mode(shape, 10.0, eps_skel=1e-10)
    assert abs(built.k - I_ref.size) <= 2
    tg = w.circle_points(31, 4.0)
    u = gs.field(shape.colloc[built.skel_idx], 10.0,
                 built.matrix64().cpu().numpy() @ (-np.exp(10j * shape.colloc[built.skel_idx][:, 1])), tg)[0]
    u_ref = gs.field(shape.colloc[I_ref], 10.0, S_ref @ (-np.exp(10j * shape.colloc[I_ref][:, 1])), tg)[0]
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-7


# ------------------------------------------------------------- scene/G_hat ---
@pytest.mark.parametrize("key", list(SMALL_SCENES))
def test_scene_packing_matches_oracle(mfs, key):
    sc = SMALL_SCENES[key]()
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    assert gsc.N == xh.shape[0] and gsc.T == sc.T
    assert np.array_equal(gsc.points(), xh)  # exact: template + centre in FP64 on both sides


@pytest.mark.parametrize("key", list(SMALL_SCENES))
@pytest.mark.parametrize("R", [1, 3])
def test_ghat_matches_oracle(mfs, key, R):
    torch = _torch()
    sc = SMALL_SCENES[key]()
    print(f"ghat parity {key} R={R}", flush=True)
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(11)
    q = crandn(rng, R, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    t64 = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t64, mfs.MFS_FP64)
    assert_entrywise(t64.cpu().numpy(), ref, 1e-12, f"G_hat FP64 {key}")
    q32 = torch.from_numpy(q.astype(np.complex64)).cuda()
    t32 = torch.empty((R, gsc.N), dtype=torch.complex64, device="cuda")
    mfs.ghat_apply(gsc, q32, t32, mfs.MFS_FP32)
    err = assert_entrywise(t32.cpu().numpy(), ref, FP32_OPERATOR_TOL, f"G_hat FP32 {key}")
    print(f"  fp32 entrywise error {err:.2e}", flush=True)


def test_single_body_has_no_pairs(mfs):
    torch = _torch()
    sc = w.make_scene("starfish2000", T=1)
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    q = torch.ones((1, gsc.N), dtype=torch.complex128, device="cuda")
    t = torch.full((1, gsc.N), 7.0, dtype=torch.complex128, device="cuda")
    mfs.ghat_apply(gsc, q, t, mfs.MFS_FP64)
    assert torch.count_nonzero(t).item() == 0


@pytest.mark.parametrize("key", ["disks16", "mixed24", "ragged9", "spheres6"])
def test_apply_matches_oracle_matvec(mfs, key):
    torch = _torch()
    sc = SMALL_SCENES[key]()
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(12)
    q = crandn(rng, 2, xh.shape[0])
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    y = torch.empty((2, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.apply(gsc, torch.from_numpy(q).cuda(), y, mfs.MFS_FP64)
    assert_entrywise(y.cpu().numpy(), ref, 1e-12, f"operator FP64 {key}")
    y32 = torch.empty((2, gsc.N), dtype=torch.complex64, device="cuda")
    mfs.apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), y32, mfs.MFS_FP32)
    assert_entrywise(y32.cpu().numpy(), ref, FP32_OPERATOR_TOL, f"operator FP32 {key}")
    # the S product alone, and b = S vhat (beta = 0)
    t = crandn(rng, 2, xh.shape[0])
    yS = torch.empty((2, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.s_apply(gsc, torch.from_numpy(q).cuda(), torch.from_numpy(t).cuda(), yS, 1.0, mfs.MFS_FP64)
    assert_entrywise(yS.cpu().numpy(), q + gs.apply_s(sc, Ss, ptr, t), 1e-13, "q + S t")
    mfs.s_apply(gsc, None, torch.from_numpy(t).cuda(), yS, 0.0, mfs.MFS_FP64)
    assert_entrywise(yS.cpu().numpy(), gs.apply_s(sc, Ss, ptr, t), 1e-13, "S t")


def test_apply_is_deterministic(mfs):
    torch = _torch()
    sc = SMALL_SCENES["mixed24"]()
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    rng = np.random.default_rng(13)
    q = torch.from_numpy(crandn(rng, 1, gsc.N)).cuda()
    ys = []
    for _ in range(2):
        y = torch.empty_like(q)
        mfs.apply(gsc, q, y, mfs.MFS_FP64)
        ys.append(y.cpu().numpy())
    assert np.array_equal(ys[0], ys[1])


def test_plane_wave_matches_oracle(mfs):
    torch = _torch()
    sc = w.make_scene("mixed2000_R64", T=16)
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    xh, _, _ = gs.pack(sc)
    v = torch.empty((sc.R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    assert_entrywise(v.cpu().numpy(), gs.plane_wave_vhat(sc, xh), 1e-13, "plane wave")


@pytest.mark.parametrize("key", ["disks16", "spheres6", "ragged9"])
def test_eval_field_matches_oracle(mfs, key):
    torch = _torch()
    sc = SMALL_SCENES[key]()
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    xh, _, _ = gs.pack(sc)
    rng = np.random.default_rng(14)
    q = crandn(rng, 2, xh.shape[0])
    tg = w.far_targets(sc, 77)
    ref = gs.field(xh, sc.kappa, q, tg)
    u = torch.empty((2, tg.shape[0]), dtype=torch.complex128, device="cuda")
    mfs.eval_field(gsc, torch.from_numpy(q).cuda(), torch.from_numpy(tg).cuda(), u, mfs.MFS_FP64)
    assert_entrywise(u.cpu().numpy(), ref, 1e-12, f"field FP64 {key}")
    u32 = torch.empty((2, tg.shape[0]), dtype=torch.complex64, device="cuda")
    mfs.eval_field(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), torch.from_numpy(tg).cuda(), u32,
                   mfs.MFS_FP32)
    assert_entrywise(u32.cpu().numpy(), ref, fp32_distance_budget(sc), f"field FP32 {key}")
    # no targets: nothing to do, no error
    empty = torch.empty((0, sc.dim), dtype=torch.float64, device="cuda")
    mfs.eval_field(gsc, torch.from_numpy(q).cuda(), empty, u, mfs.MFS_FP64)


# -------------------------------------------------------------------- solve ---
def test_solve_fp64_disks16_matches_dense_lu(mfs):
    torch = _torch()
    sc = w.make_scene("disks16")
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    v = torch.empty((1, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-10, restart=200, prec=mfs.MFS_FP64)
    assert info["relres_max"] <= 1e-10
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    assert rel_err(q.cpu().numpy(), ref) < 1e-9
    # independent residual check with the oracle operator
    b = gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh))
    r = b - gs.matvec(sc, Ss, xh, ptr, bo, q.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-10


def test_solve_fp64_with_restarts_and_multiple_rhs(mfs):
    torch = _torch()
    sc = w.make_scene("disks16")
    sc.directions = w.plane_wave_directions_2d([0.0, 1.0, 2.5])
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    v = torch.empty((3, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-10, restart=20, maxit=2000, prec=mfs.MFS_FP64)
    assert info["n_restart"] > 1 and info["relres_max"] <= 1e-10
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)))
    for c in range(3):
        assert rel_err(q.cpu().numpy()[c], ref[c]) < 1e-9


@pytest.mark.parametrize("key", ["starfish32", "spheres6", "mixed24"])
def test_solve_mixed_reaches_fp64_residual(mfs, key):
    torch = _torch()
    sc = SMALL_SCENES[key]()
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    v = torch.empty((1, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions[:1], v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, restart=200, inner_tol=1e-4, prec=mfs.MFS_MIXED)
    assert info["relres_max"] <= 1e-8 and info["n_matvec32"] > 0
    b = gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)[:1])
    r = b - gs.matvec(sc, Ss, xh, ptr, bo, q.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-8
    ref = gs.dense_solve(sc, Ss, xh, ptr, bo, b)
    tg = w.far_targets(sc, 40)
    u = gs.field(xh, sc.kappa, q.cpu().numpy(), tg)
    u_ref = gs.field(xh, sc.kappa, ref, tg)
    assert np.abs(u - u_ref).max() / np.abs(u_ref).max() < 1e-6


# ------------------------------------------------------------- edge cases ---
def test_invalid_arguments_are_rejected(mfs):
    torch = _torch()
    sc = w.make_scene("disks16", T=4)
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    q = torch.zeros((1, gsc.N), dtype=torch.complex128, device="cuda")
    with pytest.raises(mfs.MfsError) as e:
        mfs.apply(gsc, q, q, mfs.MFS_FP64)  # aliasing
    assert e.value.code == -1
    with pytest.raises(mfs.MfsError):
        mfs.solve(gsc, q, torch.empty_like(q), prec=mfs.MFS_FP32)
    with pytest.raises(mfs.MfsError):
        mfs.Scene(2, 5.0, np.array([0, 3], np.int32), np.zeros((2, 2)), [sc.shapes[0].eqpts],
                  [gsc._S_hold[0][0]])
    with pytest.raises(mfs.MfsError):
        mfs.Scene(2, -1.0, np.array([0], np.int32), np.zeros((1, 2)), [sc.shapes[0].eqpts], [gsc._S_hold[0][0]])


def test_solve_warm_start_resumes(mfs):
    """use_x0: from the converged solution no iteration is needed; from a partial solve (iteration
    cap) the resumed solve reaches the same answer as an uninterrupted one."""
    torch = _torch()
    sc = SMALL_SCENES["starfish32"]()
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    v = torch.empty((1, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q_full = torch.empty_like(v)
    mfs.solve(gsc, v, q_full, tol=1e-10, restart=500, prec=mfs.MFS_FP64)
    q = torch.empty_like(v)
    part = mfs.solve(gsc, v, q, tol=1e-10, restart=500, maxit=20, prec=mfs.MFS_FP64, raise_on_noconv=False)
    assert part["status"] == "MFS_ERR_NOCONV" and part["relres_max"] > 1e-10
    res = mfs.solve(gsc, v, q, tol=1e-10, restart=500, prec=mfs.MFS_FP64, use_x0=True)
    assert res["relres_max"] <= 1e-10
    assert rel_err(q.cpu().numpy(), q_full.cpu().numpy()) < 1e-8
    again = mfs.solve(gsc, v, q, tol=1e-10, restart=500, prec=mfs.MFS_FP64, use_x0=True)
    assert again["n_matvec64"] == 1 and again["relres_max"] <= 1e-10  # residual check only


@pytest.mark.parametrize("key", ["mixed24", "spheres6", "starfish32", "ragged9"])
@pytest.mark.parametrize("R", [16, 20, 64])
def test_ghat_many_rhs_matches_oracle(mfs, key, R):
    """R >= 8 with every body a multiple of 16 points can take the matrix-core kernel (mixed,
    spheres, starfish; R = 20 leaves a partial 64-RHS tile); up to 32 right-hand sides the symmetric
    kernel is the default where it applies, so the matrix-core kernel is also forced; ragged bodies
    stay on the plain VALU kernel."""
    torch = _torch()
    sc = SMALL_SCENES[key]()
    print(f"many-RHS G_hat {key} R={R}", flush=True)
    gsc, _ = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(31)
    q = crandn(rng, R, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    for forced in (False, True):
        if forced:
            if mfs.tune_get(gsc, R, mfs.MFS_FP32)["symmetric"] == 0:
                break
            mfs.tune_set(gsc, R, mfs.MFS_FP32, 4, 0, 0)  # the matrix-core kernel
        t32 = torch.empty((R, gsc.N), dtype=torch.complex64, device="cuda")
        mfs.ghat_apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), t32, mfs.MFS_FP32)
        got = t32.cpu().numpy()
        # every entry of every right-hand side, relative to its own right-hand side's size
        assert_entrywise(got, ref, FP32_OPERATOR_TOL, f"many-RHS G_hat {key} R={R} forced={forced}")


def test_solve_many_rhs_mixed(mfs):
    torch = _torch()
    sc = SMALL_SCENES["mixed24"]()
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    R = 16
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions[:R], v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, restart=400, inner_tol=1e-6, prec=mfs.MFS_MIXED)
    assert info["relres_max"] <= 1e-8
    b = gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)[:R])
    r = b - gs.matvec(sc, Ss, xh, ptr, bo, q.cpu().numpy())
    for c in range(R):
        assert np.linalg.norm(r[c]) / np.linalg.norm(b[c]) < 2e-8


# --------------------------------------------------------------- graph replay ---
@pytest.mark.parametrize("prec_name,restart", [("MFS_FP64", 70), ("MFS_MIXED", 150)])
def test_solve_graph_replay_is_identical_to_direct_launches(mfs, prec_name, restart):
    """Replayed graphs (bucket of 64 steps, step index on the device) run the same kernels on the
    same data as direct launches, with eager operator work between replays: results are bitwise
    equal.  restart = 70 crosses a bucket boundary and restarts several times, so graphs are
    replayed across cycles with different tolerances; two graph solves in a row must agree too."""
    torch = _torch()
    sc = SMALL_SCENES["starfish32"]()
    sc.directions = w.plane_wave_directions_2d([0.2, 1.3, 2.9])
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    v = torch.empty((3, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    prec = getattr(mfs, prec_name)
    out = []
    for use_graph in (False, True, True):
        q = torch.empty_like(v)
        info = mfs.solve(gsc, v, q, tol=1e-9, restart=restart, maxit=5000, inner_tol=1e-5, prec=prec,
                         use_graph=use_graph)
        torch.cuda.synchronize()
        assert info["relres_max"] <= 1e-9
        out.append((q.cpu().numpy(), info))
    if prec_name == "MFS_FP64":
        assert out[0][1]["n_restart"] > 1
    for q, info in out[1:]:
        assert np.array_equal(q, out[0][0])
        assert info["n_matvec32"] == out[0][1]["n_matvec32"] and info["n_matvec64"] == out[0][1]["n_matvec64"]


@pytest.mark.parametrize("key,R", [("starfish32", 1), ("mixed24", 16), ("spheres6", 2)])
def test_solve_mixed_with_single_precision_basis(mfs, key, R):
    """basis32: Krylov vectors stored in complex64, everything else as in the mixed solve; the
    final residual is still checked with the FP64 operator, here recomputed by the oracle."""
    torch = _torch()
    sc = SMALL_SCENES[key]()
    if sc.directions.shape[0] < R:
        sc.directions = w.plane_wave_directions_2d(np.linspace(0.1, 6.0, R)) if sc.dim == 2 else \
            np.tile(sc.directions[:1], (R, 1))
    gsc, Ss = _scene_with_oracle_S(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions[:R], v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, restart=300, inner_tol=3e-6, prec=mfs.MFS_MIXED, basis32=True)
    assert info["relres_max"] <= 1e-8
    b = gs.rhs(sc, Ss, ptr, gs.plane_wave_vhat(sc, xh)[:R])
    r = b - gs.matvec(sc, Ss, xh, ptr, bo, q.cpu().numpy())
    for c in range(R):
        assert np.linalg.norm(r[c]) / np.linalg.norm(b[c]) < 2e-8
