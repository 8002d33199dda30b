"""The launch-shape autotuner on the GPU: tuning picks among shapes of the same operator, so the
tuned operator still matches the FP64 oracle to the precision's tolerance, a fixed shape is
reproducible, the right-hand-sides-per-thread variants agree column by column, and scenes without
their own entry pick up the process-wide table."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, crandn, entrywise_err, make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


@pytest.fixture
def mfs(gpu_lib):
    gpu_lib.tune_clear()
    yield gpu_lib
    gpu_lib.tune_clear()  # later tests get the heuristic shapes again


def _torch():
    import torch

    return torch


def _scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


def _apply(mfs, gsc, q, prec):
    torch = _torch()
    dt = torch.complex64 if prec == mfs.MFS_FP32 else torch.complex128
    qd = torch.from_numpy(q.astype(np.complex64 if prec == mfs.MFS_FP32 else np.complex128)).cuda()
    y = torch.empty(q.shape, dtype=dt, device="cuda")
    mfs.apply(gsc, qd, y, prec)
    return y.cpu().numpy()


@pytest.mark.parametrize("prec_name", ["MFS_FP32", "MFS_FP64"])
def test_tuned_operator_matches_oracle(mfs, prec_name):
    prec = getattr(mfs, prec_name)
    sc = w.make_scene("starfish2000", T=48)
    gsc, Ss = _scene(mfs, sc)
    print(f"autotune starfish48 {prec_name}", flush=True)
    res = mfs.autotune(gsc, R=1, prec=prec, reps=2)
    assert res["n_tried"] >= 2 and res["ms"] <= res["ms_heuristic"] and res["uses_mfma"] == 0
    got = mfs.tune_get(gsc, 1, prec)
    assert got["source"] == "scene" and got["nchunks"] == res["nchunks"]
    assert mfs.tune_table_size() == 1
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(21), 1, xh.shape[0])
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    y = _apply(mfs, gsc, q, prec)
    assert entrywise_err(y, ref) < (FP32_OPERATOR_TOL if prec == mfs.MFS_FP32 else 1e-12)
    assert np.array_equal(y, _apply(mfs, gsc, q, prec))  # a fixed shape is reproducible
    # another scene with N in the same power-of-two bracket takes the table's shape
    other, _ = _scene(mfs, w.make_scene("starfish2000", T=40))
    got2 = mfs.tune_get(other, 1, prec)
    assert got2["source"] == "table" and got2["nchunks"] == res["nchunks"]
    other.close()
    gsc.close()


def test_mixed_tuning_and_rhs_per_thread_variants(mfs):
    sc = w.make_scene("mixed2000_R64", T=20)
    sc.directions = sc.directions[:3]
    gsc, Ss = _scene(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    R = 3
    print("autotune mixed20 R=3", flush=True)
    res = mfs.autotune(gsc, R=R, prec=mfs.MFS_MIXED, reps=2)
    assert res["rhs_per_thread"] in (1, 2, 4) and res["uses_mfma"] == 0
    assert res["n_tried"] >= 3  # at least the three right-hand-side groupings
    q = crandn(np.random.default_rng(22), R, xh.shape[0])
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    assert entrywise_err(_apply(mfs, gsc, q, mfs.MFS_FP32), ref) < FP32_OPERATOR_TOL
    # with the slice count fixed, grouping 1, 2 or 4 right-hand sides per thread changes which thread
    # does a column's work, not its arithmetic
    outs = []
    for rt in (1, 2, 4):
        mfs.tune_set(gsc, R, mfs.MFS_FP32, 6, rt, 0)  # the plain kernel
        assert mfs.tune_get(gsc, R, mfs.MFS_FP32) == {"nchunks": 6, "rhs_per_thread": rt, "symmetric": 0,
                                                      "source": "scene"}
        outs.append(_apply(mfs, gsc, q, mfs.MFS_FP32))
        assert entrywise_err(outs[-1], ref) < FP32_OPERATOR_TOL
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-6 * np.abs(outs[0]).max()
    mfs.tune_set(gsc, R, mfs.MFS_FP32, 0)  # back to the table entry
    assert mfs.tune_get(gsc, R, mfs.MFS_FP32)["source"] == "table"
    with pytest.raises(mfs.MfsError):
        mfs.tune_set(gsc, R, mfs.MFS_FP32, 5000)
    with pytest.raises(mfs.MfsError):
        mfs.tune_set(gsc, R, mfs.MFS_FP32, 4, 3)
    gsc.close()


def test_matrix_core_kernel_tuning(mfs):
    sc = w.make_scene("mixed2000_R64", T=16)
    sc.directions = sc.directions[:16]
    gsc, Ss = _scene(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    print("autotune mixed16 R=16 (matrix cores or symmetric)", flush=True)
    res = mfs.autotune(gsc, R=16, prec=mfs.MFS_FP32, reps=2)
    # 16 right-hand sides: the matrix-core kernel (tiles of 64) against the symmetric VALU kernel
    assert res["uses_mfma"] + res["symmetric"] == 1 and res["ms_plain"] > 0
    q = crandn(np.random.default_rng(23), 16, xh.shape[0])
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    assert entrywise_err(_apply(mfs, gsc, q, mfs.MFS_FP32), ref) < FP32_OPERATOR_TOL
    for sym in (0, 1):
        mfs.tune_set(gsc, 16, mfs.MFS_FP32, 4, 0, sym)
        got = mfs.tune_get(gsc, 16, mfs.MFS_FP32)
        assert got["symmetric"] == sym and (got["rhs_per_thread"] == 0) == (sym == 0)
        assert entrywise_err(_apply(mfs, gsc, q, mfs.MFS_FP32), ref) < FP32_OPERATOR_TOL
    print("autotune mixed16:", res, flush=True)
    gsc.close()


def test_solve_after_tuning(mfs):
    """A mixed-precision solve with tuned shapes still reaches the FP64 residual and the oracle."""
    torch = _torch()
    sc = w.make_scene("starfish2000", T=24)
    gsc, Ss = _scene(mfs, sc)
    mfs.autotune(gsc, R=1, prec=mfs.MFS_MIXED, reps=1)
    mfs.autotune(gsc, R=1, prec=mfs.MFS_FP64, reps=1)
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
    gsc.close()
