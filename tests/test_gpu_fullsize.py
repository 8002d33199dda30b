"""Full-size parity: the workloads at their real sizes, in the launch configuration the benchmark
uses, checked on sampled rows that the oracle computes one by one (each row is a sum over all N
sources), plus bilinear symmetry at full size, and the full 1000-sphere mixed-precision solve (the
benchmark's own step) checked by the oracle's FP64 residual on whole sampled bodies."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, assert_entrywise, crandn, make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


def _full_scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


@pytest.mark.parametrize("key,R", [("starfish2000", 1), ("spheres1000", 1), ("mixed2000_R64", 4),
                                   ("mixed2000_R64", 64)])
def test_full_size_ghat_sampled_rows(gpu_lib, key, R):
    """R = 64 on the mixed scene is the benchmark's many-right-hand-side configuration (the
    matrix-core kernel); R = 1 on the single-shape scenes and R = 4 take the symmetric kernel."""
    import torch

    mfs = gpu_lib
    sc = w.make_scene(key)
    print(f"full-size sampled rows: {key} N={sc.N} R={R}", flush=True)
    gsc, _ = _full_scene(mfs, sc)
    shape = mfs.tune_get(gsc, R, mfs.MFS_FP32)
    assert shape["symmetric"] == (1 if R <= 4 else 0)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(21)
    q = crandn(rng, R, sc.N)
    rows = np.sort(rng.choice(sc.N, size=24, replace=False))
    rows[0] = 0
    rows[-1] = sc.N - 1  # both ends of the packed order
    ref = gs.ghat_apply(xh, bo, sc.kappa, q, rows=rows)
    if R <= 4:
        t64 = torch.empty((R, sc.N), dtype=torch.complex128, device="cuda")
        mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t64, mfs.MFS_FP64)
        assert_entrywise(t64.cpu().numpy()[:, rows], ref, 1e-12, f"{key} FP64 rows")
    t32 = torch.empty((R, sc.N), dtype=torch.complex64, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), t32, mfs.MFS_FP32)
    err32 = assert_entrywise(t32.cpu().numpy()[:, rows], ref, FP32_OPERATOR_TOL, f"{key} FP32 rows R={R}")
    print(f"  fp32 entrywise error {err32:.3e} (tolerance {FP32_OPERATOR_TOL:.0e})", flush=True)
    # property at any size: sum_i a_i (G b)_i = sum_i b_i (G a)_i (G_hat symmetric)
    a = crandn(rng, 1, sc.N)
    b = crandn(rng, 1, sc.N)
    ta = torch.empty((1, sc.N), dtype=torch.complex128, device="cuda")
    tb = torch.empty_like(ta)
    mfs.ghat_apply(gsc, torch.from_numpy(a).cuda(), ta, mfs.MFS_FP64)
    mfs.ghat_apply(gsc, torch.from_numpy(b).cuda(), tb, mfs.MFS_FP64)
    lhs = np.sum(a * tb.cpu().numpy())
    rhs = np.sum(b * ta.cpu().numpy())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    gsc.close()


def test_full_size_spheres_mixed_solve_checked_by_oracle(gpu_lib):
    """The benchmark step's solve (1000 spheres, N = 400,000; FP32 pair sums inside FP64 GMRES with
    FP64 refinement, complex64 basis, deflated correction solves) to 1e-8.  The oracle then forms the
    FP64 residual b - (q + S G_hat q) on five whole bodies from the GPU's q (each row a sum over all
    400,000 sources): it must be small relative to each body's b, and equal, entry by entry, to the
    residual the GPU's own FP64 operator gives on those rows."""
    import torch

    mfs = gpu_lib
    sc = w.make_scene("spheres1000")
    print(f"full-size mixed solve: {sc.name} N={sc.N}", flush=True)
    gsc, Ss = _full_scene(mfs, sc)
    S = Ss[0]
    v = torch.empty((1, sc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, maxit=60000, restart=2000, max_refine=20, inner_tol=3e-6,
                     prec=mfs.MFS_MIXED, basis32=True, deflate=True)
    print(f"  solve: {info}", flush=True)
    assert info["relres_max"] <= 1e-8
    # the GPU's FP64 residual vector
    y = torch.empty_like(v)
    mfs.apply(gsc, q, y, mfs.MFS_FP64)
    bg = torch.empty_like(v)
    mfs.s_apply(gsc, None, v, bg, 0.0, mfs.MFS_FP64)
    r_gpu = (bg - y).cpu().numpy()[0]
    qh = q.cpu().numpy()
    xh, ptr, bo = gs.pack(sc)
    vhat = gs.plane_wave_vhat(sc, xh)
    bodies = [0, 137, 500, 862, sc.T - 1]
    rows = np.concatenate([np.arange(ptr[t], ptr[t + 1]) for t in bodies])
    gq = gs.ghat_apply(xh, bo, sc.kappa, qh, rows=rows)[0]
    off = 0
    for t in bodies:
        sl = slice(ptr[t], ptr[t + 1])
        k = ptr[t + 1] - ptr[t]
        b_t = S @ vhat[0, sl]
        r_t = b_t - (qh[0, sl] + S @ gq[off:off + k])
        off += k
        rel = np.linalg.norm(r_t) / np.linalg.norm(b_t)
        gap = np.abs(r_t - r_gpu[sl]).max() / np.abs(b_t).max()
        print(f"  body {t}: oracle relres {rel:.2e}, |r_oracle - r_gpu| / max|b| {gap:.2e}", flush=True)
        assert rel <= 1e-7
        assert gap <= 1e-11
    gsc.close()
