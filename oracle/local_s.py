"""Local (per-shape) construction of the scattering matrix S (Sec. 4).

Matrices, all built from phi_kappa (eq. FundamentalSol):
  A(i,j)     = phi(x_i - y_j)      m x n   MFS collocation matrix (Sec. 3.1, Sec. 4.3)
  B(i,j)     = phi(z_i - x_j)      p x m   outgoing, boundary -> proxy (eq. B-matrix)
  D(i,j)     = phi(z_i - y_j)      p x n   MFS sources -> proxy (Sec. 4.4)
  B_hat(i,j) = phi(z_i - xhat_j)   p x k   equivalent points -> proxy

Two modes are implemented.

Paper mode (Sec. 4.2-4.5): the equivalent points are a skeleton of the
collocation points chosen by column-pivoted QR of B, stopped at relative
precision eps_skel.  The ID gives Z* (k x m) with Z*[:, I] = identity and
Z*[:, rest] = R11^{-1} R12 (eq. B_fac); U = conj(Z); C solves B C = D in the
truncated least-squares sense; S = Z* C A^+ U (eq. scattering-matrix).

Given-point mode: the equivalent points xhat are supplied (for instance on a
circle just outside the body).  The same three steps are taken with B_hat in
place of the skeleton columns B(:, I):
  outgoing compression  qhat = B_hat^+ (B q)        (replaces Z* in Sec. 4.4)
  incoming interpolation w = B^T (B_hat^T)^+ what   (replaces U in Sec. 4.2)
so S = (B_hat^+ D) A^+ (B_hat^+ B)^T, using (M^T)^+ = (M^+)^T.  When xhat is
the paper's skeleton this reduces to the paper's formula: B = B_hat Z* gives
B_hat^+ B = Z* and B_hat^+ D = Z* B^+ D = Z* C.

Pseudo-inverses are truncated SVDs with relative cutoff eps_ls (Sec. 2.3 and
Sec. 3.1 allow either a truncated SVD or QR).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fundamental import phi_matrix


def local_matrices(shape, kappa: float) -> dict:
    """A, B, D and B_hat for one shape discretisation (body frame)."""
    x, y, z, xh = shape.colloc, shape.src, shape.proxy, shape.eqpts
    return dict(
        A=phi_matrix(x, y, kappa),
        B=phi_matrix(z, x, kappa),
        D=phi_matrix(z, y, kappa),
        Bh=phi_matrix(z, xh, kappa),
    )


def tsvd_solve(M: np.ndarray, rhs: np.ndarray, eps: float) -> np.ndarray:
    """Truncated-SVD least-squares solution X = M^+_eps rhs.

    Singular values <= eps * sigma_1 are dropped.  The pseudo-inverse is applied
    factor by factor, V (diag(1/s) (U^H rhs)), and never formed as a matrix:
    forming it explicitly loses about cond(M) * machine-epsilon to cancellation.
    """
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    keep = s > eps * s[0]
    coef = (U[:, keep].conj().T @ rhs) / s[keep].reshape((-1,) + (1,) * (rhs.ndim - 1))
    return Vh[keep].conj().T @ coef


def s_given_points(shape, kappa: float, eps_ls: float = 1e-13, mats: dict | None = None):
    """S = (B_hat^+ D) A^+ (B_hat^+ B)^T for supplied equivalent points."""
    M = mats if mats is not None else local_matrices(shape, kappa)
    Vstar = tsvd_solve(M["Bh"], M["D"], eps_ls)   # k x n: MFS sources -> equivalent sources
    U = tsvd_solve(M["Bh"], M["B"], eps_ls).T     # m x k: values at xhat -> boundary values
    return Vstar @ tsvd_solve(M["A"], U, eps_ls)


def interpolative_decomposition(B: np.ndarray, eps_skel: float, k_cap: int | None = None):
    """Column ID of B from column-pivoted QR (Sec. 4.2, eq. B_fac).

    Returns (I_hat, Zstar) with B ~= B[:, I_hat] @ Zstar, Zstar k x m,
    Zstar[:, I_hat] = identity.  The rank k is the number of diagonal entries
    of R with |R_jj| > eps_skel |R_11|, capped at k_cap.
    """
    Q, R, P = sla.qr(B, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    k = int(np.sum(d > eps_skel * d[0]))
    if k_cap is not None:
        k = min(k, k_cap)
    m = B.shape[1]
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])  # R11^{-1} R12
    Zstar = np.zeros((k, m), dtype=np.complex128)
    Zstar[:, P[:k]] = np.eye(k)
    Zstar[:, P[k:]] = T
    return P[:k].copy(), Zstar


def s_paper_mode(shape, kappa: float, eps_skel: float = 1e-10, eps_ls: float = 1e-13,
                 k_cap: int | None = None):
    """Paper-mode S = Z* C A^+ U with skeleton chosen by CPQR of B.

    Returns (S, I_hat).  The equivalent points are shape.colloc[I_hat].
    """
    M = local_matrices(shape, kappa)
    I_hat, Zstar = interpolative_decomposition(M["B"], eps_skel, k_cap)
    U = Zstar.T                     # conj(Z) where Z = (Z*)^H
    C = tsvd_solve(M["B"], M["D"], eps_ls)  # m x n, B C = D
    return Zstar @ C @ tsvd_solve(M["A"], U, eps_ls), I_hat


def effective_charges_from_boundary(shape, kappa: float, v_colloc: np.ndarray,
                                    eps_ls: float = 1e-13) -> np.ndarray:
    """Given-point mode analogue of S v_hat = Z* C A^+ v (Sec. 4.5, last display).

    Applies (B_hat^+ D) A^+ directly to Dirichlet data sampled on the
    collocation points instead of going through the equivalent points.
    """
    M = local_matrices(shape, kappa)
    return tsvd_solve(M["Bh"], M["D"] @ tsvd_solve(M["A"], v_colloc, eps_ls), eps_ls)
