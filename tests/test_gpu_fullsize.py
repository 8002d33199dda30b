"""Full-size parity: the workloads at their real sizes, in the launch configuration the benchmark
uses, checked on sampled rows that the oracle computes one by one (each row is a sum over all N
sources), plus the FP64 residual of a mixed-precision solve on a reduced body count."""

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import crandn, fp32_matvec_budget, make_gpu_scene, rel_err, s_to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("key", ["starfish2000", "spheres1000", "mixed2000_R64"])
def test_full_size_ghat_sampled_rows(gpu_lib, key):
    import torch

    mfs = gpu_lib
    sc = w.make_scene(key)
    print(f"full-size sampled rows: {key} N={sc.N}", flush=True)
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    xh, ptr, bo = gs.pack(sc)
    R = 4 if key == "mixed2000_R64" else 1
    rng = np.random.default_rng(21)
    q = crandn(rng, R, sc.N)
    rows = np.sort(rng.choice(sc.N, size=24, replace=False))
    rows[0] = 0
    rows[-1] = sc.N - 1  # both ends of the packed order
    ref = gs.ghat_apply(xh, bo, sc.kappa, q, rows=rows)
    t64 = torch.empty((R, sc.N), dtype=torch.complex128, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q).cuda(), t64, mfs.MFS_FP64)
    got64 = t64.cpu().numpy()[:, rows]
    assert rel_err(got64, ref) < 1e-12
    t32 = torch.empty((R, sc.N), dtype=torch.complex64, device="cuda")
    mfs.ghat_apply(gsc, torch.from_numpy(q.astype(np.complex64)).cuda(), t32, mfs.MFS_FP32)
    got32 = t32.cpu().numpy()[:, rows]
    err32 = rel_err(got32, ref)
    print(f"  fp32 rel err {err32:.3e} (budget {fp32_matvec_budget(sc):.3e})", flush=True)
    assert err32 < fp32_matvec_budget(sc)
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
