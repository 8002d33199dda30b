"""The matrix-core pair sum for many right-hand sides with FP16 products of split operands: parity
with the oracle's G_hat on scenes whose point counts leave ragged tiles and tiles that straddle
bodies, with right-hand sides of very different scales, beside the FP32 matrix-core kernel, through
the static-scratch entry point, and the scenes where it must not run."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, assert_entrywise, crandn, entrywise_err, make_gpu_scene, s_to_device
from workloads.scenes import Scene
from workloads.shapes import disk2d

pytestmark = pytest.mark.gpu

# entrywise difference between the split FP16 and the FP32 matrix-core kernels on the same FP32 phi
SPLIT_VS_FP32_TOL = 2e-6


@pytest.fixture(scope="module")
def mfs(gpu_lib):
    return gpu_lib


def _torch():
    import torch

    return torch


def _ghat_scene(mfs, sc):
    """A scene for the pair sum alone: identity S (G_hat does not read S)."""
    devs = [s_to_device(np.eye(s.k, dtype=np.complex128)) for s in sc.shapes]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc


def _ragged_2d(T=25):
    """The four mixed 2D shapes plus an 80-point disk (5 x 16 points) on every third body: nine
    such bodies, so N % 32 = 16 (a half-empty last tile) and 32-source tiles straddle bodies."""
    base = w.make_scene("mixed2000_R64", T=T)
    disk80 = disk2d(radius=0.65, m=128, n=64, src_radius=0.455, k=80, rho_eq=0.70, p=129, r_psi=0.75)
    shapes = list(base.shapes) + [disk80]
    shape_of = base.shape_of.copy()
    shape_of[::3] = len(shapes) - 1
    return Scene(2, base.kappa, shapes, shape_of.astype(np.int32), base.centres, base.directions, name="ragged2d")


CASES = {
    "ragged2d": _ragged_2d,
    "mixed24": lambda: w.make_scene("mixed2000_R64", T=24),
    "spheres5": lambda: w.make_scene("spheres1000", T=5),  # 3D, N = 2000: N % 32 = 16
}


def _ghat32(mfs, gsc, q):
    torch = _torch()
    t = torch.empty(q.shape, dtype=torch.complex64, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), t, mfs.MFS_FP32)
    return t.cpu().numpy()


@pytest.mark.parametrize("case,R", [("ragged2d", 8), ("ragged2d", 64), ("ragged2d", 70), ("mixed24", 64),
                                    ("spheres5", 64)])
def test_split_matrix_core_matches_oracle(mfs, case, R):
    sc = CASES[case]()
    print(f"split matrix-core parity {case} N={sc.N} R={R}", flush=True)
    gsc = _ghat_scene(mfs, sc)
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 3, 0, 0)  # three source slices, never the symmetric kernel
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F16X3
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(71 + R), R, sc.N).astype(np.complex64).astype(np.complex128)
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    t16 = _ghat32(mfs, gsc, q)
    t16b = _ghat32(mfs, gsc, q)
    mfs.set_split_fp16(gsc, False)
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F32
    t32 = _ghat32(mfs, gsc, q)
    mfs.set_split_fp16(gsc, True)
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F16X3
    err16, err32, between = entrywise_err(t16, ref), entrywise_err(t32, ref), entrywise_err(t16, t32)
    print(f"  entrywise error: split FP16 {err16:.2e}, FP32 {err32:.2e}, between the two {between:.2e}", flush=True)
    assert np.array_equal(t16b, t16)  # deterministic
    assert err16 <= FP32_OPERATOR_TOL and err32 <= FP32_OPERATOR_TOL
    # both kernels evaluate the same FP32 phi, so their difference is the split operands' and the
    # accumulation order's alone: ~2^-21 per product
    assert between <= SPLIT_VS_FP32_TOL
    gsc.close()


def test_split_matrix_core_column_scales(mfs):
    """Each right-hand side is scaled by its own power of two before the split: columns from 1e-30
    to 1e30, a zero column (exact zeros out), a column with one non-zero entry, and a column whose
    entries span twenty decades, each held to the tolerance relative to its own largest entry."""
    sc = _ragged_2d()
    R = 12
    print(f"split matrix-core column scales N={sc.N} R={R}", flush=True)
    gsc = _ghat_scene(mfs, sc)
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 2, 0, 0)
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F16X3
    rng = np.random.default_rng(5)
    q = crandn(rng, R, sc.N)
    for c, s in enumerate([1e-30, 1e-12, 1e-3, 1.0, 1e3, 1e12, 1e30]):
        q[c] *= s
    q[7] = 0.0
    q[8] = 0.0
    q[8, sc.N // 3] = 2.5 - 1.0j
    q[9] *= 10.0 ** rng.uniform(-20, 0, sc.N)
    q[10] = q[10].real  # imaginary parts all zero
    q = q.astype(np.complex64).astype(np.complex128)
    xh, ptr, bo = gs.pack(sc)
    got = _ghat32(mfs, gsc, q)
    assert np.all(got[7] == 0)
    nz = [c for c in range(R) if c != 7]
    ref = gs.ghat_apply(xh, bo, sc.kappa, q[nz])
    err = assert_entrywise(got[nz], ref, FP32_OPERATOR_TOL, "column scales")
    print(f"  entrywise error {err:.2e}", flush=True)
    gsc.close()


def test_close_bodies_keep_fp32_matrix_cores(mfs):
    """3D bodies whose equivalent-point spheres reach into each other give no bound on |phi|: the
    FP32 matrix-core kernel runs, and asking for the split form is an error.  The FP32 distance of
    the body-centre split, r^2 = D^2 + u, cancels for points much closer than their centres:
    relative error ~2^-24 (D / r_min)^2, which sets the tolerance here."""
    sc = w.make_scene("spheres1000", T=3)
    sc.centres = np.array([[0.0, 0.0, 0.0], [2.1, 0.0, 0.0], [0.0, 5.0, 0.0]])
    R = 16
    print(f"close 3D bodies N={sc.N} R={R}", flush=True)
    gsc = _ghat_scene(mfs, sc)
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 2, 0, 0)
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F32
    with pytest.raises(mfs.MfsError):
        mfs.set_split_fp16(gsc, True)
    xh, ptr, bo = gs.pack(sc)
    a, b = xh[bo == 0], xh[bo == 1]
    r_min = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1)).min()
    tol = max(FP32_OPERATOR_TOL, 20 * 2.0 ** -24 * (2.1 / r_min) ** 2)
    q = crandn(np.random.default_rng(9), R, sc.N).astype(np.complex64).astype(np.complex128)
    err = assert_entrywise(_ghat32(mfs, gsc, q), gs.ghat_apply(xh, bo, sc.kappa, q), tol, "close bodies")
    print(f"  r_min {r_min:.3f}, entrywise error {err:.2e} (tolerance {tol:.1e})", flush=True)
    gsc.close()


def test_split_matrix_core_operator_and_static_entry(mfs):
    """The operator q + S G_hat q with 64 right-hand sides: mfs_apply and mfs_apply_static (split
    charges after the partial slices in the static array) against the oracle."""
    torch = _torch()
    sc = w.make_scene("mixed2000_R64", T=24)
    R = 64
    print(f"operator with split matrix cores N={sc.N} R={R}", flush=True)
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP32) == mfs.MFS_PAIR_MC_F16X3
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(12), R, sc.N).astype(np.complex64).astype(np.complex128)
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    qd = torch.from_numpy(q.astype(np.complex64)).cuda()
    y = torch.empty_like(qd)
    mfs.apply(gsc, qd, y, mfs.MFS_FP32)
    e1 = assert_entrywise(y.cpu().numpy(), ref, FP32_OPERATOR_TOL, "apply")
    ys = torch.full_like(qd, 3.0)
    mfs.apply_static(gsc, qd, ys, mfs.MFS_FP32)
    e2 = assert_entrywise(ys.cpu().numpy(), ref, FP32_OPERATOR_TOL, "apply_static")
    print(f"  apply {e1:.2e}, apply_static {e2:.2e}, between {entrywise_err(ys.cpu().numpy(), y.cpu().numpy()):.2e}",
          flush=True)
    gsc.close()


@pytest.mark.parametrize("case,R", [("ragged2d", 8), ("ragged2d", 70), ("spheres5", 64)])
def test_fp64_matrix_core_matches_oracle(mfs, case, R):
    """The FP64 pair sum with 8 or more right-hand sides runs on the FP64 matrix cores (phi once per
    pair for 64 right-hand sides): the oracle's G_hat q to 1e-12, entry by entry."""
    torch = _torch()
    sc = CASES[case]()
    print(f"FP64 matrix-core parity {case} N={sc.N} R={R}", flush=True)
    gsc = _ghat_scene(mfs, sc)
    assert mfs.pair_kernel(gsc, R, mfs.MFS_FP64) == mfs.MFS_PAIR_MC_F64
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(81 + R), R, sc.N)
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    t = torch.empty((R, sc.N), dtype=torch.complex128, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t, mfs.MFS_FP64)
    err = assert_entrywise(t.cpu().numpy(), ref, 1e-12, f"FP64 matrix cores {case}")
    print(f"  entrywise error {err:.2e}", flush=True)
    gsc.close()
