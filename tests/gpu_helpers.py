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


def fp32_matvec_budget(sc) -> float:
    """Error model for the FP32 operator: 10 (kappa L + 10) 2^-24, L the scene diameter."""
    return 10.0 * (sc.kappa * 2.0 * sc.radius() + 10.0) * 2.0 ** -24
