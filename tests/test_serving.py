"""Serving loop on the CPU: admission by footprint, slots, FIFO order and failure handling with a
fake executor (no device).  The GPU test runs the same engine on real requests and checks that
each result is the same alone and in the mix."""

import threading
import time

import numpy as np
import pytest

import workloads as w
from paper_2603_19113_amd.serve import Admission, Engine, footprint_bytes, latency_stats, replay, restart_for


class FakeExecutor:
    def __init__(self, engine_ref, durations):
        self.engine_ref = engine_ref
        self.durations = durations
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.max_used = 0
        self.order = []

    def __call__(self, spec, slot):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.max_used = max(self.max_used, self.engine_ref[0].policy.used)
            self.order.append(spec.rid)
        time.sleep(self.durations[spec.rid])
        with self.lock:
            self.active -= 1
        if spec.rid == 3:
            raise RuntimeError("injected failure")
        return {"rid": spec.rid, "slot": slot}


class Spec:
    def __init__(self, rid, arrival=0.0):
        self.rid = rid
        self.arrival = arrival


def test_admission_policy_bounds():
    a = Admission(budget=100, slots=2)
    assert a.fits(60)
    a.admit(60)
    assert not a.fits(50)        # budget
    assert a.fits(40)
    a.admit(40)
    assert not a.fits(1)         # slots and budget
    a.release(60)
    assert a.fits(50) and a.running == 1
    with pytest.raises(ValueError):
        a.fits(101)


def test_engine_respects_budget_slots_and_fifo():
    rng = np.random.default_rng(0)
    n = 12
    fps = [int(x) for x in rng.integers(10, 60, size=n)]
    ref = [None]
    ex = FakeExecutor(ref, durations=[0.02 + 0.01 * (i % 3) for i in range(n)])
    eng = Engine(ex, budget=100, slots=3)
    ref[0] = eng
    specs = [Spec(i) for i in range(n)]
    for s, fp in zip(specs, fps):
        eng.submit(s, fp)
    assert eng.drain(timeout=30)
    eng.close()
    assert ex.max_active <= 3
    assert ex.max_used <= 100
    assert ex.order == sorted(ex.order)          # admitted in arrival order
    tk = {t.rid: t for t in eng.tickets}
    assert tk[3].error is not None and "injected" in tk[3].error
    assert all(tk[i].error is None and tk[i].result["rid"] == i for i in range(n) if i != 3)
    assert eng.policy.used == 0 and eng.policy.running == 0
    st = latency_stats(eng.tickets)
    assert st["n"] == n - 1 and st["failed"] == 1 and st["p99_s"] >= st["p50_s"] > 0


def test_engine_rejects_oversized_request():
    eng = Engine(lambda s, slot: {}, budget=10, slots=1)
    with pytest.raises(ValueError):
        eng.submit(Spec(0), 11)
    eng.close()


def test_replay_follows_arrivals():
    ref = [None]
    ex = FakeExecutor(ref, durations=[0.005] * 4)
    eng = Engine(ex, budget=10, slots=2)
    ref[0] = eng
    specs = [Spec(i, arrival=0.02 * i) for i in range(3)]
    tickets = replay(eng, specs, [1, 1, 1])
    eng.close()
    arr = [t.arrival for t in tickets]
    assert arr == sorted(arr) and arr[2] - arr[0] >= 0.03


def test_request_stream_is_seeded_and_shaped():
    a = w.serving.request_stream(6, rate=2.0, seed=5, t_min=3, t_max=12)
    b = w.serving.request_stream(6, rate=2.0, seed=5, t_min=3, t_max=12)
    for x, y in zip(a, b):
        assert x.arrival == y.arrival and x.scene.T == y.scene.T and np.array_equal(x.scene.centres, y.scene.centres)
    assert all(3 <= s.scene.T <= 12 and 1 <= s.scene.R <= 16 for s in a)
    assert [s.arrival for s in a] == sorted(s.arrival for s in a)


def test_footprint_grows_with_size_and_basis():
    small = footprint_bytes(1000, 10, 1, 2, restart_for(10, 10.0, 2))
    large = footprint_bytes(64000, 500, 4, 2, restart_for(500, 10.0, 2))
    assert 0 < small < large
    assert restart_for(5000, 20.0, 2) == 4000  # capped
