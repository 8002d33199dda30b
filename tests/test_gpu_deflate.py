"""Deflated correction solves (GCRO over the first inner solve's Krylov space) through the C ABI:
the answer meets the tolerance under the oracle's own residual, it needs fewer FP32 operator
applications than correction solves that restart from scratch, graph replay of the first inner
solve changes nothing, several right-hand sides keep spaces of their own lengths, a column that is
already converged is left alone, and a basis workspace with no room left falls back to the plain
refinement bit for bit."""

import dataclasses

import numpy as np
import pytest

import workloads as w
from oracle import global_system as gs, local_s
from tests.gpu_helpers import make_gpu_scene, s_to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfs(gpu_lib):
    return gpu_lib


@pytest.fixture(scope="module")
def starfish64(mfs):
    sc = w.make_scene("starfish2000", T=64)
    Ss = [local_s.s_given_points(s, sc.kappa) for s in sc.shapes]
    devs = [s_to_device(S) for S in Ss]
    gsc = make_gpu_scene(mfs, sc, [d[0] for d in devs], [d[1] for d in devs])
    gsc._S_hold = devs
    return sc, Ss, gsc


def _solve(mfs, gsc, sc, R, zero_col=None, **kw):
    import torch

    dirs = w.plane_wave_directions_2d(np.linspace(0.2, 5.0, R))
    v = torch.empty((R, gsc.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(gsc, dirs, v)
    if zero_col is not None:
        v[zero_col].zero_()
    q = torch.empty_like(v)
    info = mfs.solve(gsc, v, q, tol=1e-8, maxit=6000, prec=mfs.MFS_MIXED, basis32=True, **kw)
    torch.cuda.synchronize()
    return q.cpu().numpy(), info, dirs


def _oracle_relres(sc, Ss, dirs, q):
    xh, ptr, bo = gs.pack(sc)
    sc2 = dataclasses.replace(sc, directions=dirs)
    b = gs.rhs(sc2, Ss, ptr, gs.plane_wave_vhat(sc2, xh))
    r = b - gs.matvec(sc2, Ss, xh, ptr, bo, q)
    return max(np.linalg.norm(r[c]) / np.linalg.norm(b[c]) for c in range(q.shape[0]))


@pytest.mark.parametrize("R", [1, 3])
def test_deflated_correction_solves_converge_with_fewer_steps(mfs, starfish64, R):
    sc, Ss, gsc = starfish64
    # a loose first inner solve, so that the correction solves carry most of the work
    plain_q, plain, dirs = _solve(mfs, gsc, sc, R, restart=2000, inner_tol=1e-4)
    defl_q, defl, _ = _solve(mfs, gsc, sc, R, restart=2000, inner_tol=1e-4, deflate=True)
    graph_q, graph, _ = _solve(mfs, gsc, sc, R, restart=2000, inner_tol=1e-4, deflate=True, use_graph=True)
    print("plain", plain, "\ndeflated", defl)
    assert plain["n_refine"] >= 2  # the correction solves are exercised
    for q, info in ((plain_q, plain), (defl_q, defl)):
        assert info["relres_max"] <= 1e-8
        assert _oracle_relres(sc, Ss, dirs, q) < 2e-8
    assert defl["n_matvec32"] < 0.9 * plain["n_matvec32"]
    # graph replay of the first inner solve: the same arithmetic, launched differently
    assert np.array_equal(graph_q, defl_q)
    assert graph["n_matvec32"] == defl["n_matvec32"] and graph["n_refine"] == defl["n_refine"]
    # the two answers differ by no more than the tolerance allows (conditioning ~ 1e2 here)
    assert np.linalg.norm(defl_q - plain_q) / np.linalg.norm(plain_q) < 1e-5


def test_deflated_solve_leaves_a_converged_column_alone(mfs, starfish64):
    """A zero right-hand side is converged from the start: it keeps no space (k = 0), takes no
    correction, and its solution stays exactly zero while the other columns are deflated."""
    sc, Ss, gsc = starfish64
    q, info, dirs = _solve(mfs, gsc, sc, 3, zero_col=1, restart=2000, inner_tol=1e-4, deflate=True)
    assert info["relres_max"] <= 1e-8 and info["n_refine"] >= 2
    assert not np.any(q[1])
    keep = [0, 2]
    assert _oracle_relres(sc, Ss, dirs[keep], q[keep]) < 2e-8


def test_deflate_without_room_falls_back_to_plain_refinement(mfs, starfish64):
    sc, Ss, gsc = starfish64
    # a workspace 30 steps longer than the first inner solve: too short to keep its space
    _, probe, _ = _solve(mfs, gsc, sc, 1, restart=2000, inner_tol=1e-4, max_refine=1, raise_on_noconv=False)
    kw = dict(restart=probe["n_matvec32"] + 30, inner_tol=1e-4)
    q0, i0, _ = _solve(mfs, gsc, sc, 1, **kw)
    q1, i1, _ = _solve(mfs, gsc, sc, 1, deflate=True, **kw)
    assert i0["relres_max"] <= 1e-8
    assert np.array_equal(q0, q1)
    assert i0["n_matvec32"] == i1["n_matvec32"] and i0["n_refine"] == i1["n_refine"]
