"""Full MFS sources of each body and the field near the bodies (Sec. 4.6 and the field formula of
Sec. 2.3).  Test infrastructure only, like the rest of this package.  Bodies may be rotated copies of
their shape (scene.rotations): every point set of the body turns with it and S, A and U, which
depend only on distances within the body, are the shape's.

After the global solve, the equivalent sources q_hat of body tau represent its scattered field only
outside its proxy surface Psi_tau.  Closer in, the paper reconstructs the body's own MFS sources
(on Gamma_tau^mfs, the curve or surface of the sources y_j):

    q_tau^mfs = A_tau^+ ( v_tau - U_tau w_hat_tau ),   w_hat_tau = (G_hat q_hat)_tau,

where v_tau is the Dirichlet data at the collocation points of Gamma_tau, w_hat_tau is the field of
all other bodies at tau's equivalent points, and U_tau interpolates it to the collocation points.
The field of body tau is then sum_j phi(x - y_j) q_j^mfs anywhere outside Gamma_tau^mfs, so the
total scattered field can be evaluated up to the boundaries: bodies whose proxy surface contains x
contribute through their MFS sources, the others through their equivalent points.

U depends on how the equivalent points were chosen (local_s): with given points
U = (B_hat^+ B)^T, in paper mode U = conj(Z).  Pseudo-inverses are truncated SVDs applied factor by
factor (local_s.tsvd_solve).
"""

from __future__ import annotations

import numpy as np

from .fundamental import phi_matrix
from .global_system import ghat_apply
from .local_s import local_matrices, tsvd_solve


def incoming_map(shape, kappa: float, eps_ls: float = 1e-13) -> np.ndarray:
    """U (m x k) for supplied equivalent points: values at x_hat -> values at the collocation points."""
    M = local_matrices(shape, kappa)
    return tsvd_solve(M["Bh"], M["B"], eps_ls).T


def collocation_offsets(scene) -> tuple[np.ndarray, np.ndarray]:
    """Start of each body's collocation points and of its MFS sources in body order."""
    m = np.array([scene.shapes[int(s)].colloc.shape[0] for s in scene.shape_of], np.int64)
    n = np.array([scene.shapes[int(s)].src.shape[0] for s in scene.shape_of], np.int64)
    return np.concatenate([[0], np.cumsum(m)]), np.concatenate([[0], np.cumsum(n)])


def plane_wave_on_boundary(scene, directions=None) -> np.ndarray:
    """v = -exp(i kappa d . x) at every body's collocation points, [R, sum m] (footnote to eq. BVP)."""
    dirs = np.atleast_2d(scene.directions if directions is None else directions)
    pts = np.concatenate([scene.place(t, scene.shapes[int(s)].colloc) for t, s in enumerate(scene.shape_of)], 0)
    return -np.exp(1j * scene.kappa * (dirs @ pts.T))


def reconstruct_mfs(scene, U_of_shape, xhat, body_of, qhat, v_colloc, eps_ls: float = 1e-13,
                    workers: int | None = None) -> np.ndarray:
    """q^mfs of every body, [R, sum n], from the solved equivalent sources (Sec. 4.6)."""
    qhat = np.atleast_2d(qhat)
    v_colloc = np.atleast_2d(v_colloc)
    w_hat = ghat_apply(xhat, body_of, scene.kappa, qhat, workers=workers)
    cptr, sptr = collocation_offsets(scene)
    kptr = np.concatenate([[0], np.cumsum([scene.shapes[int(s)].eqpts.shape[0] for s in scene.shape_of])])
    out = np.zeros((qhat.shape[0], sptr[-1]), np.complex128)
    A_of_shape = [phi_matrix(s.colloc, s.src, scene.kappa) for s in scene.shapes]
    for t, s in enumerate(scene.shape_of):
        s = int(s)
        rhs = v_colloc[:, cptr[t]:cptr[t + 1]] - w_hat[:, kptr[t]:kptr[t + 1]] @ U_of_shape[s].T
        out[:, sptr[t]:sptr[t + 1]] = tsvd_solve(A_of_shape[s], rhs.T, eps_ls).T
    return out


def field_near(scene, xhat, qhat, q_mfs, targets) -> np.ndarray:
    """Scattered field at targets anywhere outside the MFS source curves/surfaces, [R, M]: body tau
    contributes through its MFS sources where the target lies inside Psi_tau (|x - c_tau| < the
    proxy radius), through its equivalent points elsewhere."""
    qhat = np.atleast_2d(qhat)
    q_mfs = np.atleast_2d(q_mfs)
    targets = np.atleast_2d(targets)
    _, sptr = collocation_offsets(scene)
    kptr = np.concatenate([[0], np.cumsum([scene.shapes[int(s)].eqpts.shape[0] for s in scene.shape_of])])
    u = np.zeros((qhat.shape[0], targets.shape[0]), np.complex128)
    for t, s in enumerate(scene.shape_of):
        sh = scene.shapes[int(s)]
        c = scene.centres[t]
        near = np.linalg.norm(targets - c[None, :], axis=1) < sh.proxy_radius
        if np.any(~near):
            u[:, ~near] += qhat[:, kptr[t]:kptr[t + 1]] @ phi_matrix(targets[~near], xhat[kptr[t]:kptr[t + 1]],
                                                                      scene.kappa).T
        if np.any(near):
            u[:, near] += q_mfs[:, sptr[t]:sptr[t + 1]] @ phi_matrix(targets[near], scene.place(t, sh.src),
                                                                      scene.kappa).T
    return u
