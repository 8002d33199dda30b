"""The block-diagonal S product on the matrix cores (16 or more right-hand sides, FP32 S): the
operator q + S G_hat q against the oracle entry by entry with the pair sums in the packed layout
(matrix-core and symmetric sub-block pair kernels) and in the padded layout (symmetric kernel on
bodies that are not whole tiles), bodies of 64 to 400 points (row tiles cut by the body size),
right-hand sides past a whole column tile (70), and mfs_s_apply with the caller's own t, which the
product only reads."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import FP32_OPERATOR_TOL, assert_entrywise, crandn, make_gpu_scene, s_to_device
from tests.test_gpu_mc16 import _ragged_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfs(gpu_lib):
    return gpu_lib


def _torch():
    import torch

    return torch


def _scene(mfs, sc):
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return gsc, Ss


CASES = {"ragged2d": _ragged_2d, "spheres5": lambda: w.make_scene("spheres1000", T=5)}


@pytest.mark.parametrize("case,R", [("ragged2d", 16), ("ragged2d", 20), ("ragged2d", 64), ("ragged2d", 70),
                                    ("spheres5", 16), ("spheres5", 64)])
def test_operator_with_matrix_core_S_product(mfs, case, R):
    torch = _torch()
    sc = CASES[case]()
    gsc, Ss = _scene(mfs, sc)
    print(f"matrix-core S product {case} N={sc.N} R={R} pair kernel "
          f"{mfs.PAIR_KERNEL_NAMES[mfs.pair_kernel(gsc, R, mfs.MFS_FP32)]}", flush=True)
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(60 + R), R, sc.N).astype(np.complex64).astype(np.complex128)
    ref = gs.matvec(sc, Ss, xh, ptr, bo, q)
    qd = torch.from_numpy(q.astype(np.complex64)).cuda()
    # the untuned kernel, then (up to 24 right-hand sides) the symmetric kernel, whose partial sums
    # on bodies that are not whole tiles sit in the padded layout
    for forced_sym in (False, True):
        if forced_sym:
            if R > 24:
                break
            mfs.tune_set(gsc, R, mfs.MFS_FP32, 3, 0, 1)
        y = torch.empty_like(qd)
        mfs.apply(gsc, qd, y, mfs.MFS_FP32)
        err = assert_entrywise(y.cpu().numpy(), ref, FP32_OPERATOR_TOL, f"operator {case} R={R} sym={forced_sym}")
        ys = torch.empty_like(qd)
        mfs.apply_static(gsc, qd, ys, mfs.MFS_FP32)
        err_s = assert_entrywise(ys.cpu().numpy(), ref, FP32_OPERATOR_TOL,
                                 f"static operator {case} R={R} sym={forced_sym}")
        print(f"  sym={forced_sym}: entrywise error {err:.2e}, static entry {err_s:.2e}", flush=True)
    gsc.close()


def test_s_apply_reads_the_callers_t(mfs):
    torch = _torch()
    sc = _ragged_2d()
    R = 16
    gsc, Ss = _scene(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(77)
    q = crandn(rng, R, sc.N).astype(np.complex64)
    t = crandn(rng, R, sc.N).astype(np.complex64)
    ref = 0.5 * q.astype(np.complex128) + gs.apply_s(sc, Ss, ptr, t.astype(np.complex128))
    qd, td = torch.from_numpy(q).cuda(), torch.from_numpy(t).cuda()
    t_before = td.clone()
    y = torch.empty_like(qd)
    mfs.s_apply(gsc, qd, td, y, 0.5, mfs.MFS_FP32)
    assert torch.equal(td, t_before)  # read only
    err = assert_entrywise(y.cpu().numpy(), ref, 1e-5, "s_apply R=16")
    print(f"s_apply entrywise error {err:.2e}", flush=True)
    gsc.close()
