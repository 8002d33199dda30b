"""Serving on the GPU: requests run one at a time and concurrently (overlapping on the device through
per-slot streams, and batched with other requests on the same geometry) give the same solutions."""

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _run(specs, slots, batching=None):
    from paper_2603_19113_amd.serve import Engine, GpuExecutor, latency_stats, request_footprint

    eng = Engine(GpuExecutor(slots), budget=16 << 30, slots=slots, batching=batching, start=False)
    for s in specs:
        eng.submit(s, request_footprint([s]))
    eng.start()
    assert eng.drain(timeout=240)
    eng.close()
    errors = [t.error for t in eng.tickets if t.error]
    assert not errors, errors
    print(f"slots={slots} batching={batching is not None}: {latency_stats(eng.tickets)}", flush=True)
    return {t.rid: t for t in eng.tickets}


def test_results_same_alone_and_in_the_mix(gpu_lib):
    specs = w.serving.request_stream(6, rate=50.0, seed=11, t_min=3, t_max=10, r_max=4)
    print("requests:", [s.scene.name for s in specs], flush=True)
    alone = _run(specs, 1)
    mix = _run(specs, 3)
    for rid, a in alone.items():
        b = mix[rid]
        assert a.result["info"]["relres_max"] <= 1e-8 and b.result["info"]["relres_max"] <= 1e-8
        # deterministic kernels and request-local arithmetic: identical, not merely close
        assert np.array_equal(a.result["qhat"], b.result["qhat"]), rid


def test_batched_requests_match_their_solo_solves(gpu_lib):
    from paper_2603_19113_amd import mfs
    from paper_2603_19113_amd.serve import request_batching

    specs = w.serving.request_stream(8, rate=50.0, seed=12, t_min=3, t_max=8, r_max=3, p_sweep=0.6)
    print("requests:", [s.scene.name for s in specs], flush=True)
    alone = _run(specs, 1)
    hits0 = mfs.pool_stats()["hits"]
    mix = _run(specs, 3, batching=request_batching())
    assert any(t.batch > 1 for t in mix.values())
    assert mfs.pool_stats()["hits"] > hits0          # Krylov bases and tables reused from the cache
    for rid, a in alone.items():
        b = mix[rid]
        qa, qb = a.result["qhat"], b.result["qhat"]
        assert qa.shape == qb.shape
        assert a.result["info"]["relres_max"] <= 1e-8 and b.result["info"]["relres_max"] <= 1e-8
        # both meet the 1e-8 residual; the systems are well conditioned, so the solutions agree to
        # far better than the 1e-6 stated for mixed-precision results
        for r in range(qa.shape[0]):
            rel = np.linalg.norm(qa[r] - qb[r]) / np.linalg.norm(qa[r])
            assert rel <= 1e-6, (rid, r, rel, b.batch)


@pytest.mark.parametrize("key,T,R", [("mixed2000_R64", 24, 64), ("starfish2000", 40, 1), ("spheres1000", 5, 3)])
def test_footprint_covers_what_a_solve_allocates(gpu_lib, key, T, R):
    """mfs_solve_footprint against the scene's own device bytes after a mixed solve (block GMRES for
    several directions, as the serving loop runs it) and an FP64 field evaluation, with the
    allocation cache emptied first so that every block is a fresh one."""
    import torch

    from paper_2603_19113_amd.serve import block_solve, restart_for

    mfs = gpu_lib
    sc = w.make_scene(key, T=T)
    sc.directions = np.resize(sc.directions, (R, sc.dim)) if sc.R != R else sc.directions
    built = [mfs.build_S(s, sc.kappa) for s in sc.shapes]
    torch.cuda.synchronize()
    mfs.pool_trim()
    scene = mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                      [b.S64 for b in built], [b.S32 for b in built])
    restart = restart_for(sc.T, sc.kappa, sc.dim, R)
    v = torch.empty((R, scene.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(scene, sc.directions, v)
    q = torch.empty_like(v)
    info = mfs.solve(scene, v, q, tol=1e-8, maxit=100000, restart=restart, max_refine=30, inner_tol=3e-6,
                     prec=mfs.MFS_MIXED, basis32=True, deflate=True, block=block_solve(R))
    tg = torch.from_numpy(np.ascontiguousarray(w.far_targets(sc, 64))).cuda()
    u = torch.empty((R, tg.shape[0]), dtype=torch.complex128, device="cuda")
    mfs.eval_field(scene, q, tg, u, mfs.MFS_FP64)
    torch.cuda.synchronize()
    held = scene.size()[2]
    est = mfs.solve_footprint(sc.dim, sc.shape_of, sc.k_of_shape, R, restart, prec=mfs.MFS_MIXED,
                              block=block_solve(R), basis32=True, n_targets=tg.shape[0])
    print(f"{key} T={T} R={R}: relres {info['relres_max']:.1e}, scene holds {held / 1e6:.1f} MB, "
          f"footprint {est / 1e6:.1f} MB", flush=True)
    assert info["relres_max"] <= 1e-8
    assert held <= est
    assert held >= 0.5 * est
    scene.close()
