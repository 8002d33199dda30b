"""The global system (I + S G_hat) qhat = S vhat (eq. mbody2) and its pieces.

Vectors are RHS-major arrays of shape [R, N] (complex128).  The equivalent
points of body tau are x_hat = template + c_tau, packed contiguously body by
body in body order (translated copies share S, Sec. 5.1 Example 4).

G_hat(i, j) = phi_kappa(xhat_i - xhat_j) when points i and j lie on different
bodies and 0 otherwise (eq. Gmtx-entries; G_hat holds only the off-diagonal
blocks, eq. mbody2).
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .fundamental import phi_matrix


# ---------------------------------------------------------------- packing ---
def pack(scene):
    """Global equivalent points, body pointer and body index of each point."""
    pts, body_of, ptr = [], [], [0]
    for tau in range(scene.T):
        s = scene.shapes[int(scene.shape_of[tau])]
        pts.append(scene.place(tau, s.eqpts))  # x_hat = R_tau template + c_tau
        body_of.append(np.full(s.k, tau, dtype=np.int64))
        ptr.append(ptr[-1] + s.k)
    return np.concatenate(pts, 0), np.asarray(ptr, np.int64), np.concatenate(body_of)


# ----------------------------------------------------------------- G_hat ----
def ghat_dense(xhat: np.ndarray, body_of: np.ndarray, kappa: float) -> np.ndarray:
    """Dense G_hat (small N only); same-body entries, including i = j, are 0."""
    G = np.zeros((xhat.shape[0], xhat.shape[0]), dtype=np.complex128)
    for i in range(xhat.shape[0]):
        other = body_of != body_of[i]
        G[i, other] = phi_matrix(xhat[i:i + 1], xhat[other], kappa)[0]
    return G


def _ghat_rows(xhat, body_of, kappa, q, rows):
    out = np.empty((q.shape[0], rows.shape[0]), dtype=np.complex128)
    for a, i in enumerate(rows):
        other = body_of != body_of[i]
        g = phi_matrix(xhat[i:i + 1], xhat[other], kappa)[0]
        out[:, a] = q[:, other] @ g
    return out


def ghat_apply(xhat, body_of, kappa, q, rows=None, workers: int | None = None, block=64):
    """t = G_hat q for q [R, N]; optionally only the listed target rows.

    Row blocks are spread over a thread pool (scipy's Hankel ufunc releases
    the interpreter lock), one row at a time inside a block.
    """
    q = np.atleast_2d(np.asarray(q, dtype=np.complex128))
    rows = np.arange(xhat.shape[0]) if rows is None else np.asarray(rows)
    # default pool: the host's cores, at most 16 (one GPU's share of a shared benchmark host)
    workers = workers or min(os.cpu_count() or 1, 16)
    chunks = [rows[s:s + block] for s in range(0, rows.shape[0], block)]
    if workers == 1 or len(chunks) == 1:
        parts = [_ghat_rows(xhat, body_of, kappa, q, c) for c in chunks]
    else:
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(lambda c: _ghat_rows(xhat, body_of, kappa, q, c), chunks))
    return np.concatenate(parts, axis=1)


# ---------------------------------------------------------- S and matvec ---
def apply_s(scene, S_of_shape, ptr, t):
    """Block-diagonal S: y_tau = S_{shape(tau)} t_tau for every body tau."""
    t = np.atleast_2d(t)
    y = np.empty_like(t)
    for tau in range(scene.T):
        a, b = ptr[tau], ptr[tau + 1]
        y[:, a:b] = (S_of_shape[int(scene.shape_of[tau])] @ t[:, a:b].T).T
    return y


def matvec(scene, S_of_shape, xhat, ptr, body_of, q, workers=None):
    """y = q + S G_hat q (the operator of eq. mbody2)."""
    q = np.atleast_2d(q)
    return q + apply_s(scene, S_of_shape, ptr, ghat_apply(xhat, body_of, scene.kappa, q,
                                                          workers=workers))


def plane_wave_vhat(scene, xhat):
    """Dirichlet data at x_hat for sound-soft bodies: v = -u_inc, u_inc = exp(i kappa d.x).

    Returns [R, N] (footnote to eq. BVP: v = -u_inc).
    """
    phase = scene.kappa * (scene.directions @ xhat.T)
    return -np.exp(1j * phase)


def rhs(scene, S_of_shape, ptr, vhat):
    """b = S vhat (right side of eq. mbody2)."""
    return apply_s(scene, S_of_shape, ptr, vhat)


def dense_operator(scene, S_of_shape, xhat, ptr, body_of):
    """I + S G_hat as a dense N x N matrix (small N only)."""
    G = ghat_dense(xhat, body_of, scene.kappa)
    N = xhat.shape[0]
    SG = np.empty_like(G)
    for tau in range(scene.T):
        a, b = ptr[tau], ptr[tau + 1]
        SG[a:b, :] = S_of_shape[int(scene.shape_of[tau])] @ G[a:b, :]
    return np.eye(N, dtype=np.complex128) + SG


def condition_number(scene, S_of_shape, xhat, ptr, body_of):
    """K = cond_2(I + S G_hat), the condition number of the global coefficient matrix of eq. mbody2
    that Sec. 5.1 (Example 1) reports: largest over smallest singular value, by a dense SVD (small N
    only)."""
    sv = np.linalg.svd(dense_operator(scene, S_of_shape, xhat, ptr, body_of), compute_uv=False)
    return float(sv[0] / sv[-1])


def dense_solve(scene, S_of_shape, xhat, ptr, body_of, b):
    """qhat = (I + S G_hat)^{-1} b by LU (numpy.linalg.solve); b [R, N]."""
    Aop = dense_operator(scene, S_of_shape, xhat, ptr, body_of)
    return np.linalg.solve(Aop, np.atleast_2d(b).T).T


def gmres(apply, b, tol=1e-12, maxit=2000):
    """Full (unrestarted) GMRES with x0 = 0 for one right-hand side b [N].

    Arnoldi with modified Gram-Schmidt and Givens rotations (Saad & Schultz
    1986); stops when the Givens residual estimate falls to tol * ||b||.
    Returns (x, iterations, relative residual estimate).
    """
    b = np.asarray(b, dtype=np.complex128)
    beta = np.linalg.norm(b)
    N = b.shape[0]
    V = np.zeros((maxit + 1, N), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit, dtype=np.complex128)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    if beta == 0.0:
        return np.zeros_like(b), 0, 0.0
    V[0] = b / beta
    g[0] = beta
    j = 0
    res = 1.0
    for j in range(maxit):
        w = apply(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] != 0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            tmp = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = tmp
        den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = np.conj(cs[j]) * g[j]
        res = abs(g[j + 1]) / beta
        if res <= tol:
            break
    k = j + 1
    yk = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    return V[:k].T @ yk, k, res


# ----------------------------------------------------------------- field ----
def field(xhat, kappa, qhat, targets):
    """u(x) = sum_j phi(x - xhat_j) qhat_j (eq. out_skel); returns [R, M]."""
    return np.atleast_2d(qhat) @ phi_matrix(targets, xhat, kappa).T


def incoming_on_body(scene, xhat, ptr, qhat, tau, points, v_points):
    """w_tau = v - sum_{sigma != tau} u_sigma at given points near body tau (eq. w_in)."""
    a, b = ptr[tau], ptr[tau + 1]
    mask = np.ones(xhat.shape[0], dtype=bool)
    mask[a:b] = False
    return v_points - field(xhat[mask], scene.kappa, np.atleast_2d(qhat)[:, mask], points)
