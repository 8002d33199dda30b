"""Free-space fundamental solution of -Delta - kappa^2 (eq. FundamentalSol).

2D: phi(x) = (i/4) H_0^(1)(kappa |x|)
3D: phi(x) = exp(i kappa |x|) / (4 pi |x|)

H_0^(1) is taken from scipy.special.hankel1 (AMOS), in float64.
"""

from __future__ import annotations

import numpy as np
import scipy.special as sp


def phi_of_r(r: np.ndarray, kappa: float, dim: int) -> np.ndarray:
    """phi_kappa as a function of the distance r > 0."""
    r = np.asarray(r, dtype=np.float64)
    if dim == 2:
        return 0.25j * sp.hankel1(0, kappa * r)
    if dim == 3:
        return np.exp(1j * kappa * r) / (4.0 * np.pi * r)
    raise ValueError("dim must be 2 or 3")


def phi_matrix(targets: np.ndarray, sources: np.ndarray, kappa: float) -> np.ndarray:
    """M(i, j) = phi_kappa(targets_i - sources_j); targets [M,d], sources [N,d]."""
    diff = targets[:, None, :] - sources[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    return phi_of_r(r, kappa, targets.shape[1])
