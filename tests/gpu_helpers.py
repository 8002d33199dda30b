"""Helpers shared by the GPU tests: build scenes from workloads through the C ABI binding."""

from __future__ import annotations

import numpy as np


def s_to_device(S: np.ndarray):
    """Upload a row-major numpy S (k x k) as column-major device storage (complex128, complex64)."""
    import torch

    colmajor = np.ascontiguousarray(S.T)
    s64 = torch.from_numpy(colmajor.astype(np.complex128)).cuda()
    s32 = torch.from_numpy(colmajor.astype(np.complex64)).cuda()
    return s64, s32


def make_gpu_scene(mfs, sc, S_list_dev64, S_list_dev32):
    return mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes], S_list_dev64,
                     S_list_dev32, rotations=getattr(sc, "rotations", None))


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# FP32 pair sums with the body-centre phase split (G_hat, the operator, the symmetric and matrix-core
# kernels): the phase kappa r is formed as kappa D (FP64, per body pair) + kappa delta (FP32, |delta|
# below two body radii), so each term carries ~1e-6 rad of phase error and ~1e-7 of amplitude error
# whatever the scene size.  Measured at full size: 6e-7 (spheres), 7e-7 (starfish), 1.3e-6 (mixed,
# kappa 20) relative to the largest entry; the bound below is about 10x that.
FP32_OPERATOR_TOL = 1e-5


def fp32_distance_budget(sc) -> float:
    """Error model of an FP32 pair sum on plain single-precision distances (field evaluation at
    external targets): 10 (kappa L + 10) 2^-24, L the scene diameter."""
    return 10.0 * (sc.kappa * 2.0 * sc.radius() + 10.0) * 2.0 ** -24


def entrywise_err(got, ref) -> float:
    """max over right-hand sides r and entries i of |got[r,i] - ref[r,i]| / max_i |ref[r,i]|: every
    entry of every right-hand side is held to the tolerance, scaled by its own row's size."""
    got = np.atleast_2d(np.asarray(got))
    ref = np.atleast_2d(np.asarray(ref))
    assert got.shape == ref.shape, (got.shape, ref.shape)
    scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)
    return float((np.abs(got - ref) / scale).max())


def assert_entrywise(got, ref, tol, what=""):
    err = entrywise_err(got, ref)
    assert err <= tol, f"{what}: entrywise error {err:.3e} > {tol:.1e}"
    return err
