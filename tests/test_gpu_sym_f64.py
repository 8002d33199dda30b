"""The FP64 symmetric pair sum (3D, one right-hand side: the refinement residual of the mixed solve)
against the FP64 oracle entry by entry: phi once per unordered pair, same-body pairs removed pair by
pair, so tiles may straddle bodies of any size.  Cases: one body (no pairs), bodies of 48, 80 and
400 points (several bodies per tile, tiles across body boundaries), two shapes, a last tile partly
filled, group counts from 1 to over 30 (with the padding of the group count to whole blocks), and the
whole operator against the plain FP64 kernel that the allocation-free entry point runs."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs
from tests.gpu_helpers import assert_entrywise, crandn, entrywise_err
from tests.test_gpu_sym import _scene, _spheres_k, _two_sphere_shapes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfs(gpu_lib):
    return gpu_lib


def _torch():
    import torch

    return torch


CASES = [("k400", 1), ("k400", 3), ("k48", 9), ("k48", 23), ("k80", 5), ("mix", 13), ("k48", 170),
         ("spheres1000", 20)]


def _make(case, T):
    if case == "mix":
        return _two_sphere_shapes(T)
    if case == "spheres1000":
        return w.make_scene("spheres1000", T=T)
    return _spheres_k(T, int(case[1:]))


@pytest.mark.parametrize("case,T", CASES)
def test_fp64_symmetric_kernel_matches_oracle(mfs, case, T):
    torch = _torch()
    sc = _make(case, T)
    sc.directions = sc.directions[:1]
    print(f"FP64 symmetric ghat {case} T={T} N={sc.N}", flush=True)
    gsc, Ss = _scene(mfs, sc)
    xh, ptr, bo = gs.pack(sc)
    q = crandn(np.random.default_rng(41 + T), 1, xh.shape[0])
    ref = gs.ghat_apply(xh, bo, sc.kappa, q)
    t = torch.empty((1, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t, mfs.MFS_FP64)
    got = t.cpu().numpy()
    if T == 1:
        assert np.count_nonzero(got) == 0
    else:
        err = assert_entrywise(got, ref, 1e-12, f"FP64 symmetric {case}")
        print(f"  entrywise error {err:.2e}", flush=True)
    t2 = torch.empty_like(t)
    mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t2, mfs.MFS_FP64)
    assert torch.equal(t, t2)  # deterministic
    # the operator: symmetric (mfs_apply) against the plain kernel (mfs_apply_static) and the oracle
    ref_y = gs.matvec(sc, Ss, xh, ptr, bo, q)
    qd = torch.from_numpy(q).cuda()
    y = torch.empty_like(qd)
    mfs.apply(gsc, qd, y, mfs.MFS_FP64)
    ys = torch.empty_like(qd)
    mfs.apply_static(gsc, qd, ys, mfs.MFS_FP64)
    assert_entrywise(y.cpu().numpy(), ref_y, 1e-12, f"operator FP64 symmetric {case}")
    between = entrywise_err(y.cpu().numpy(), ys.cpu().numpy())
    print(f"  symmetric against plain kernel {between:.2e}", flush=True)
    assert between <= 1e-13
    gsc.close()
