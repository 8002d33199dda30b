"""mfs_apply_static, the operator y = q + S G_hat q with every intermediate in the library's static
per-device scratch array (for callers that cannot allocate), against mfs_apply on the same inputs,
through the C ABI: two calls in a row, the second with a smaller input; neither allocates."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, assert_entrywise, crandn, make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


def _scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


def _alloc_state(mfs, torch):
    torch.cuda.synchronize()
    p = mfs.pool_stats()
    return (p["hits"], p["misses"], p["live_bytes"], torch.cuda.memory_allocated())


@pytest.mark.parametrize("prec_name", ["MFS_FP32", "MFS_FP64"])
def test_apply_static_matches_apply_twice_then_smaller(gpu_lib, prec_name):
    """First call: 600 starfish (N = 76,800), where the symmetric kernel's slices (~130 MB) exceed
    the 64 MiB array, so the FP32 call runs the plain kernel with the slices that fit.  Second
    call, smaller: 12 spheres (400 points, padded to whole tiles for the symmetric kernel, whose
    padded charges also go into the array) with three right-hand sides, also checked against the
    oracle.  The allocation cache's counters and torch's allocated bytes must not move."""
    import torch

    mfs = gpu_lib
    prec = getattr(mfs, prec_name)
    ctype = torch.complex64 if prec == mfs.MFS_FP32 else torch.complex128
    tol = FP32_OPERATOR_TOL if prec == mfs.MFS_FP32 else 1e-12
    cases = [(w.make_scene("starfish2000", T=600), 1), (w.make_scene("spheres1000", T=12), 3)]
    for i, (sc, R) in enumerate(cases):
        print(f"apply_static call {i}: {sc.name} N={sc.N} R={R} {prec_name}", flush=True)
        gsc, Ss = _scene(mfs, sc)
        q = torch.from_numpy(crandn(np.random.default_rng(40 + i), R, sc.N)).to(ctype).cuda()
        y_ref = torch.empty_like(q)
        mfs.apply(gsc, q, y_ref, prec)
        y = torch.full_like(q, 7.0)  # stale values must not leak into the result
        before = _alloc_state(mfs, torch)
        mfs.apply_static(gsc, q, y, prec)
        after = _alloc_state(mfs, torch)
        assert after == before, (before, after)
        got = y.cpu().numpy()
        err = assert_entrywise(got, y_ref.cpu().numpy(), tol, f"static vs apply, call {i}")
        print(f"  static vs apply: entrywise {err:.2e}", flush=True)
        if sc.N <= 5000:
            xh, ptr, bo = gs.pack(sc)
            ref = gs.matvec(sc, Ss, xh, ptr, bo, q.cpu().numpy().astype(np.complex128))
            assert_entrywise(got, ref, tol, f"static vs oracle, call {i}")
        gsc.close()


def test_apply_static_rejects_what_does_not_fit(gpu_lib):
    """One partial slice of R x N complex64 beyond 64 MiB: a clear MFS_ERR_ARG, nothing enqueued,
    the output left untouched."""
    import torch

    mfs = gpu_lib
    sc = w.make_scene("starfish2000", T=600)
    gsc, _ = _scene(mfs, sc)
    R = 128  # 128 x 76,800 x 8 bytes = 78.6 MB > 64 MiB
    assert R * sc.N * 8 > mfs.STATIC_SCRATCH_BYTES
    q = torch.zeros((R, sc.N), dtype=torch.complex64, device="cuda")
    y = torch.full_like(q, 3.0)
    with pytest.raises(mfs.MfsError) as e:
        mfs.apply_static(gsc, q, y, mfs.MFS_FP32)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 3.0).all())
    gsc.close()
