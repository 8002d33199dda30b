"""Serving on the GPU: the same requests run one at a time and concurrently (overlapping on the
device through per-slot streams) give the same solutions, each to the solve tolerance."""

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_the_mix(gpu_lib):
    from paper_2603_19113_amd.serve import Engine, GpuExecutor, footprint_bytes, latency_stats, restart_for

    specs = w.serving.request_stream(6, rate=50.0, seed=11, t_min=3, t_max=10, r_max=4)
    fps = [footprint_bytes(s.scene.N, s.scene.T, s.scene.R, s.scene.dim,
                           restart_for(s.scene.T, s.scene.kappa, s.scene.dim)) for s in specs]
    print("requests:", [s.scene.name for s in specs], flush=True)
    results = {}
    for slots in (1, 3):
        ex = GpuExecutor(slots)
        eng = Engine(ex, budget=8 << 30, slots=slots)
        for s, fp in zip(specs, fps):
            eng.submit(s, fp)
        assert eng.drain(timeout=240)
        eng.close()
        errors = [t.error for t in eng.tickets if t.error]
        assert not errors, errors
        results[slots] = {t.rid: t.result for t in eng.tickets}
        st = latency_stats(eng.tickets)
        print(f"slots={slots}: {st}", flush=True)
    for rid in results[1]:
        a, b = results[1][rid], results[3][rid]
        assert a["info"]["relres_max"] <= 1e-8 and b["info"]["relres_max"] <= 1e-8
        # deterministic kernels and request-local arithmetic: identical, not merely close
        assert np.array_equal(a["qhat"], b["qhat"]), rid
