"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, a series solution of the
same boundary value problem, an independent library (mpmath), brute force on
tiny inputs, or a structural invariant of the method.  Comments give the
measured error at the time the tolerance was set.
"""

import mpmath
import numpy as np
import pytest

import workloads as w
from oracle import fundamental, global_system as gs, local_s
from tests.analytic import MultiDisk, disk_series, graf_check, mie_series


# ------------------------------------------------------------- phi_kappa ----
def test_phi_2d_matches_mpmath_hankel():
    rng = np.random.default_rng(1)
    z = 10.0 ** rng.uniform(-6, np.log10(3000.0), size=300)
    got = fundamental.phi_of_r(z, 1.0, 2)
    mpmath.mp.dps = 30
    for zi, gi in zip(z, got):
        ref = complex(0.25j * mpmath.hankel1(0, mpmath.mpf(float(zi))))
        assert abs(gi - ref) <= 2e-14 * abs(ref)


def test_phi_3d_matches_closed_form_mpmath():
    rng = np.random.default_rng(2)
    r = 10.0 ** rng.uniform(-4, 2.5, size=200)
    kappa = 3.0
    got = fundamental.phi_of_r(r, kappa, 3)
    mpmath.mp.dps = 30
    for ri, gi in zip(r, got):
        R = mpmath.mpf(float(ri))
        ref = complex(mpmath.exp(1j * kappa * R) / (4 * mpmath.pi * R))
        # the phase kappa r carries ~ulp(kappa r) absolute error in float64
        assert abs(gi - ref) <= 2.2e-16 * (8 + 2 * kappa * ri) * abs(ref)


# ---------------------------------------------------- single-body physics ---
@pytest.mark.parametrize("alpha", [0.0, 0.7])
def test_single_disk_given_points_matches_series(alpha):
    """T = 1: G_hat = 0, so qhat = S vhat; its field must be the disk series."""
    shape = w.c1_disks16().shapes[0]
    kappa = 5.0
    S = local_s.s_given_points(shape, kappa)
    d = np.array([np.cos(alpha), np.sin(alpha)])
    vhat = -np.exp(1j * kappa * shape.eqpts @ d)
    tg = w.circle_points(37, 2.5, 0.3)
    u = gs.field(shape.eqpts, kappa, S @ vhat, tg)[0]
    ref = disk_series(kappa, 1.0, alpha, tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-10  # measured 4.5e-12


def test_single_disk_paper_mode_matches_series():
    """Paper mode: skeleton from CPQR of B (Sec. 4.2), S = Z* C A^+ U."""
    shape = w.disk2d(radius=1.0, m=128, n=64, src_radius=0.7, k=64, rho_eq=1.2, p=128, r_psi=1.5)
    kappa = 5.0
    S, I_hat = local_s.s_paper_mode(shape, kappa, eps_skel=1e-12)
    xh = shape.colloc[I_hat]
    vhat = -np.exp(1j * kappa * xh[:, 0])
    tg = w.circle_points(29, 2.5, 0.1)
    u = gs.field(xh, kappa, S @ vhat, tg)[0]
    ref = disk_series(kappa, 1.0, 0.0, tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-9


def test_paper_mode_equals_given_mode_on_its_skeleton():
    """With xhat = Gamma(I_hat), the given-point formula reduces to Z* C A^+ U."""
    shape = w.starfish2d(m=192, n=96, d=0.1, k=60, rho_eq=0.67, p=193, r_psi=1.5,
                         r0=81 / 101, amp=-20 / 81)
    kappa = 10.0
    S_p, I_hat = local_s.s_paper_mode(shape, kappa, eps_skel=1e-10)
    skel = w.ShapeDiscretisation("skel", 2, shape.colloc, shape.src, shape.proxy,
                                 shape.colloc[I_hat], shape.bounding_radius, shape.proxy_radius)
    S_g = local_s.s_given_points(skel, kappa)
    # compare actions on a smooth incoming field (plane wave) through the far field
    vhat = -np.exp(1j * kappa * skel.eqpts[:, 1])
    tg = w.circle_points(31, 4.0)
    u_p = gs.field(skel.eqpts, kappa, S_p @ vhat, tg)[0]
    u_g = gs.field(skel.eqpts, kappa, S_g @ vhat, tg)[0]
    assert np.abs(u_p - u_g).max() / np.abs(u_g).max() < 1e-7


def test_paper_starfish_skeleton_size_is_plausible():
    """Soft check (parity unpinned): the paper's starfish at kappa = 10, eps 1e-10
    reports 54 skeleton points; the proxy radius is not given, so only a range."""
    shape = w.starfish2d(m=256, n=128, d=0.1, k=128, rho_eq=0.67, p=257, r_psi=1.5,
                         r0=81 / 101, amp=-20 / 81)
    _, I_hat = local_s.s_paper_mode(shape, 10.0, eps_skel=1e-10)
    assert 35 <= I_hat.size <= 90


def test_single_starfish_matches_fine_plain_mfs():
    """S built on the starfish discretisation vs a 4x finer classical MFS solve
    (least squares on 1024 collocation points, 512 sources)."""
    shape = w.c2_starfish2000(T=4).shapes[0]
    kappa = 10.0
    S = local_s.s_given_points(shape, kappa)
    fine = w.starfish2d(m=1024, n=512, d=0.06)
    A = fundamental.phi_matrix(fine.colloc, fine.src, kappa)
    tg = w.circle_points(41, 3.0, 0.2)
    for alpha in (0.0, 1.3):
        d = np.array([np.cos(alpha), np.sin(alpha)])
        q_fine = np.linalg.lstsq(A, -np.exp(1j * kappa * fine.colloc @ d), rcond=1e-14)[0]
        ref = fundamental.phi_matrix(tg, fine.src, kappa) @ q_fine
        u = gs.field(shape.eqpts, kappa, S @ (-np.exp(1j * kappa * shape.eqpts @ d)), tg)[0]
        assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-7  # measured 5.5e-9


def test_single_sphere_matches_mie_series():
    sc = w.c3_spheres1000(T=1)
    shape = sc.shapes[0]
    S = local_s.s_given_points(shape, sc.kappa)
    vhat = -np.exp(1j * sc.kappa * shape.eqpts[:, 0])
    tg = w.fibonacci_sphere(50, 3.0)
    u = gs.field(shape.eqpts, sc.kappa, S @ vhat, tg)[0]
    ref = mie_series(sc.kappa, 1.0, [1.0, 0.0, 0.0], tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-5  # measured 2.4e-6


def test_disk_S_is_circulant_and_symmetric():
    """Rotational symmetry of the disk (m, n, p multiples of k) makes S circulant;
    reciprocity of phi makes it complex-symmetric."""
    shape = w.c1_disks16().shapes[0]
    S = local_s.s_given_points(shape, 5.0)
    k = S.shape[0]
    for s in range(1, k, 7):
        assert np.allclose(np.roll(np.roll(S, s, 0), s, 1), S, rtol=0, atol=1e-9 * abs(S).max())
    assert np.linalg.norm(S - S.T) / np.linalg.norm(S) < 1e-8  # measured 1.8e-10


def test_effective_charges_from_boundary_data_agree():
    """S vhat (values at xhat) vs applying B_hat^+ D A^+ to v on Gamma (Sec. 4.5)."""
    shape = w.c1_disks16().shapes[0]
    kappa = 5.0
    d = np.array([np.cos(0.4), np.sin(0.4)])
    S = local_s.s_given_points(shape, kappa)
    a = S @ (-np.exp(1j * kappa * shape.eqpts @ d))
    b = local_s.effective_charges_from_boundary(shape, kappa, -np.exp(1j * kappa * shape.colloc @ d))
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-8


# ------------------------------------------------------ multibody physics ---
def test_graf_addition_theorem_numerically():
    lhs, rhs = graf_check(5.0, 3, np.array([0.0, 0.0]), np.array([3.0, 0.5]),
                          np.array([3.4, 0.9]))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_sixteen_disks_match_multipole_solution():
    sc = w.c1_disks16()
    S = local_s.s_given_points(sc.shapes[0], sc.kappa)
    xh, ptr, bo = gs.pack(sc)
    b = gs.rhs(sc, [S], ptr, gs.plane_wave_vhat(sc, xh))
    q = gs.dense_solve(sc, [S], xh, ptr, bo, b)
    tg = w.far_targets(sc, 64)
    u = gs.field(xh, sc.kappa, q, tg)[0]
    ref = MultiDisk(sc.kappa, 1.0, sc.centres, 0.0, nmax=25).field(tg)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-9  # measured 8.8e-12


def test_incoming_field_on_a_disk_matches_multipole():
    """E_inc: w_tau = v - sum_{sigma != tau} u_sigma on Gamma_tau (eq. w_in)."""
    sc = w.c1_disks16(T=4)
    S = local_s.s_given_points(sc.shapes[0], sc.kappa)
    xh, ptr, bo = gs.pack(sc)
    q = gs.dense_solve(sc, [S], xh, ptr, bo, gs.rhs(sc, [S], ptr, gs.plane_wave_vhat(sc, xh)))
    md = MultiDisk(sc.kappa, 1.0, sc.centres, 0.0, nmax=25)
    tau = 3
    pts = sc.centres[tau] + w.circle_points(50, 1.0, 0.5)
    v = -np.exp(1j * sc.kappa * pts[:, 0])
    got = gs.incoming_on_body(sc, xh, ptr, q, tau, pts, v)[0]
    # reference: v minus the other disks' multipole fields
    ref = v.copy()
    for j, c in enumerate(md.centres):
        if j == tau:
            continue
        sub = MultiDisk.__new__(MultiDisk)
        sub.kappa, sub.centres, sub.modes = md.kappa, c[None, :], md.modes
        sub.coef = md.coef[j:j + 1]
        ref -= sub.field(pts)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-9


# --------------------------------------------------- brute force on G_hat ---
def test_matvec_bruteforce_tiny_mpmath():
    """Three bodies (two shapes), random S and q; every entry by hand with mpmath."""
    rng = np.random.default_rng(3)
    sh = [w.ShapeDiscretisation("a", 2, np.zeros((1, 2)), np.zeros((1, 2)), np.zeros((1, 2)),
                                rng.normal(size=(2, 2)) * 0.3, 1.0, 1.0),
          w.ShapeDiscretisation("b", 2, np.zeros((1, 2)), np.zeros((1, 2)), np.zeros((1, 2)),
                                rng.normal(size=(3, 2)) * 0.3, 1.0, 1.0)]
    sc = w.Scene(dim=2, kappa=2.5, shapes=sh, shape_of=np.array([1, 0, 1], np.int32),
                 centres=np.array([[0.0, 0.0], [4.0, 1.0], [-1.0, 5.0]]),
                 directions=np.array([[1.0, 0.0]]))
    S_of = [rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)),
            rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))]
    xh, ptr, bo = gs.pack(sc)
    q = rng.normal(size=(1, 8)) + 1j * rng.normal(size=(1, 8))
    got = gs.matvec(sc, S_of, xh, ptr, bo, q, workers=1)[0]
    mpmath.mp.dps = 25
    pts, body = [], []
    for tau, s in enumerate(sc.shape_of):
        for e in sh[s].eqpts:
            pts.append(e + sc.centres[tau])
            body.append(tau)
    t = []
    for i in range(8):
        acc = 0j
        for j in range(8):
            if body[i] != body[j]:
                r = float(np.hypot(*(pts[i] - pts[j])))
                acc += complex(0.25j * mpmath.hankel1(0, sc.kappa * r)) * q[0, j]
        t.append(acc)
    t = np.array(t)
    ref = q[0].copy()
    for tau, s in enumerate(sc.shape_of):
        a, b = ptr[tau], ptr[tau + 1]
        ref[a:b] += S_of[s] @ t[a:b]
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("key", ["disks16", "spheres1000"])
def test_ghat_bilinear_symmetry_single_body_and_translation(key):
    sc = w.make_scene(key, T=4 if key == "disks16" else 3)
    xh, ptr, bo = gs.pack(sc)
    rng = np.random.default_rng(4)
    a = rng.normal(size=xh.shape[0]) + 1j * rng.normal(size=xh.shape[0])
    b = rng.normal(size=xh.shape[0]) + 1j * rng.normal(size=xh.shape[0])
    Ga = gs.ghat_apply(xh, bo, sc.kappa, a)[0]
    Gb = gs.ghat_apply(xh, bo, sc.kappa, b)[0]
    assert abs(a @ Gb - b @ Ga) < 1e-12 * abs(a @ Gb)
    # one body: no off-body pairs
    one = np.zeros_like(bo)
    assert np.abs(gs.ghat_apply(xh, one, sc.kappa, a)).max() == 0.0
    # translating every point leaves G_hat unchanged
    shift = np.full(xh.shape[1], 17.25)
    Ga2 = gs.ghat_apply(xh + shift, bo, sc.kappa, a)[0]
    assert np.abs(Ga2 - Ga).max() < 1e-11 * np.abs(Ga).max()


def test_gmres_matches_dense_lu():
    sc = w.c1_disks16()
    S = local_s.s_given_points(sc.shapes[0], sc.kappa)
    xh, ptr, bo = gs.pack(sc)
    b = gs.rhs(sc, [S], ptr, gs.plane_wave_vhat(sc, xh))
    q = gs.dense_solve(sc, [S], xh, ptr, bo, b)[0]
    x, it, res = gs.gmres(lambda z: gs.matvec(sc, [S], xh, ptr, bo, z)[0], b[0], tol=1e-12)
    assert res <= 1e-12
    assert np.linalg.norm(x - q) / np.linalg.norm(q) < 1e-10  # measured 2.9e-12
    # the true residual of the dense solution
    r = b[0] - gs.matvec(sc, [S], xh, ptr, bo, q)[0]
    assert np.linalg.norm(r) / np.linalg.norm(b[0]) < 1e-13


def _one_point_scene(dim, kappa, centres):
    """Bodies of one equivalent point each (the body centre), for closed forms of I + S G_hat."""
    z = np.zeros((1, dim))
    sh = w.ShapeDiscretisation(name="point", dim=dim, colloc=z, src=z, proxy=z, eqpts=z, bounding_radius=0.0,
                               proxy_radius=0.0)
    c = np.asarray(centres, np.float64)
    return w.Scene(dim=dim, kappa=kappa, shapes=[sh], shape_of=np.zeros(c.shape[0], np.int32), centres=c,
                   directions=np.array([[1.0] + [0.0] * (dim - 1)]))


def test_condition_number_of_one_body_is_one():
    """One body: G_hat has no off-body entries, so I + S G_hat = I and K = 1 for any S."""
    sc = w.make_scene("disks16", T=1)
    S = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    xh, ptr, bo = gs.pack(sc)
    assert abs(gs.condition_number(sc, S, xh, ptr, bo) - 1.0) < 1e-12


@pytest.mark.parametrize("dim,kappa,d,s", [(2, 3.0, 1.7, 0.8 - 0.3j), (3, 2.0, 0.9, -1.1 + 0.4j),
                                           (2, 10.0, 0.25, 2.0 + 1.0j)])
def test_condition_number_two_point_bodies_closed_form(dim, kappa, d, s):
    """Two one-point bodies a distance d apart with S = [s]: I + S G_hat = [[1, c], [c, 1]],
    c = s phi(d), a normal matrix with eigenvalues 1 +- c, so K = max |1 +- c| / min |1 +- c|."""
    sc = _one_point_scene(dim, kappa, [[0.0] * dim, [d] + [0.0] * (dim - 1)])
    xh, ptr, bo = gs.pack(sc)
    K = gs.condition_number(sc, [np.array([[s]])], xh, ptr, bo)
    r = float(d)
    phi = (0.25j * complex(mpmath.hankel1(0, kappa * r)) if dim == 2
           else complex(mpmath.exp(1j * kappa * r)) / (4.0 * np.pi * r))
    c = s * phi
    a, b = abs(1 + c), abs(1 - c)
    assert abs(K - max(a, b) / min(a, b)) < 1e-12 * max(a, b) / min(a, b)


def test_condition_number_three_point_bodies_in_extended_precision():
    """Three one-point bodies on a line with S = [s] (I + S G_hat is no longer normal): K against the
    square root of the extreme eigenvalues of M^H M, with M formed entry by entry from mpmath's
    Hankel function and the eigenvalues taken by mpmath in extended precision."""
    kappa, s = 4.0, 0.9 + 0.2j
    sc = _one_point_scene(2, kappa, [[0.0, 0.0], [0.8, 0.0], [1.9, 0.0]])
    xh, ptr, bo = gs.pack(sc)
    K = gs.condition_number(sc, [np.array([[s]])], xh, ptr, bo)
    M = np.eye(3, dtype=complex)
    for i in range(3):
        for j in range(3):
            if i != j:
                M[i, j] = s * 0.25j * complex(mpmath.hankel1(0, kappa * abs(xh[i, 0] - xh[j, 0])))
    # singular values from the eigenvalues of M^H M, by mpmath in extended precision
    ev = mpmath.eigh(mpmath.matrix((M.conj().T @ M).tolist()), eigvals_only=True)
    ev = sorted(float(mpmath.re(e)) for e in ev)
    assert K >= 1.0
    assert abs(K - np.sqrt(ev[-1] / ev[0])) < 1e-10 * K
