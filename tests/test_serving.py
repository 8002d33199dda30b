"""Serving loop on the CPU: admission by footprint, slots, FIFO order and failure handling with a
fake executor (no device).  The GPU test runs the same engine on real requests and checks that
each result is the same alone and in the mix."""

import threading
import time

import numpy as np
import pytest

import workloads as w
from paper_2603_19113_amd.serve import (Admission, Batching, Engine, footprint_bytes, latency_stats, replay,
                                        request_footprint, restart_for)


class FakeExecutor:
    def __init__(self, engine_ref, durations):
        self.engine_ref = engine_ref
        self.durations = durations
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.max_used = 0
        self.order = []
        self.batches = []

    def __call__(self, specs, slot):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.max_used = max(self.max_used, self.engine_ref[0].policy.used)
            self.order.extend(s.rid for s in specs)
            self.batches.append([s.rid for s in specs])
        time.sleep(max(self.durations[s.rid] for s in specs))
        with self.lock:
            self.active -= 1
        if any(s.rid == 3 for s in specs):
            raise RuntimeError("injected failure")
        return [{"rid": s.rid, "slot": slot, "batch": len(specs)} for s in specs]


class Spec:
    def __init__(self, rid, arrival=0.0, geometry=None, R=1):
        self.rid = rid
        self.arrival = arrival
        self.geometry = rid if geometry is None else geometry
        self.R = R


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
    tk = {t.rid: t for t in eng.tickets}
    assert [tk[i].admitted for i in range(n)] == list(range(n))   # admitted in arrival order
    assert tk[3].error is not None and "injected" in tk[3].error
    assert all(tk[i].error is None and tk[i].result["rid"] == i for i in range(n) if i != 3)
    assert eng.policy.used == 0 and eng.policy.running == 0
    st = latency_stats(eng.tickets)
    assert st["n"] == n - 1 and st["failed"] == 1 and st["p99_s"] >= st["p50_s"] > 0


def test_engine_rejects_oversized_request():
    eng = Engine(lambda specs, slot: [{} for _ in specs], budget=10, slots=1)
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
    small = footprint_bytes(2, np.zeros(10, np.int32), [100], 1, restart_for(10, 10.0, 2))
    large = footprint_bytes(2, np.zeros(500, np.int32), [128], 4, restart_for(500, 10.0, 2, 4))
    assert 0 < small < large
    assert restart_for(5000, 20.0, 2) == 4000  # capped
    assert restart_for(5000, 20.0, 2, R=8) == 2000  # block steps, capped
    assert restart_for(2000, 20.0, 2, R=64) >= 687  # the full-size mixed scene's measured block steps
    assert restart_for(495, 5.0, 2, R=8) >= 500     # 125 stalled there (30 restarted cycles at 4e-7)


def test_footprint_comes_from_the_library():
    """The estimate is the library's (mfs_solve_footprint) plus the caller's vectors: it counts the
    symmetric kernel's partial slices up to 32 right-hand sides (about N/512 per right-hand side on
    bodies padded to 64-point tiles), the block basis for several directions, and grows with R."""
    from paper_2603_19113_amd import mfs

    shape_of = (np.arange(256) % 2).astype(np.int32)
    ks = [112, 144]                     # not multiples of 64: the symmetric kernel's padded layout
    N = 128 * 256
    lib16 = mfs.solve_footprint(2, shape_of, ks, 16, 200, block=True, basis32=True)
    assert footprint_bytes(2, shape_of, ks, 16, 200) == lib16 + 2 * 16 * N * 16 + 16 * 16
    n_pad = 128 * 128 + 192 * 128       # 112 -> 128 and 144 -> 192 points
    slices = 2 * n_pad // 512           # at least the source-side slices per right-hand side
    assert lib16 >= slices * 16 * n_pad * 8
    # a longer basis and more right-hand sides cost more; block and per-column bases differ
    assert mfs.solve_footprint(2, shape_of, ks, 16, 400, block=True, basis32=True) > lib16
    assert mfs.solve_footprint(2, shape_of, ks, 1, 200, basis32=True) < lib16
    with pytest.raises(mfs.MfsError):
        mfs.solve_footprint(2, shape_of, ks, 65, 200, block=True)   # the block solve takes <= 64


def test_batching_merges_same_geometry_within_rhs_cap():
    # slot 0 busy with request 0; then 1..6 queue up: geometries 7,7,8,7,7,7 with R = 3 each
    ref = [None]
    durations = [0.15] + [0.01] * 6
    ex = FakeExecutor(ref, durations)
    b = Batching(key=lambda s: s.geometry, rhs=lambda s: s.R, footprint=lambda specs: 10 + sum(s.R for s in specs),
                 max_rhs=9)
    eng = Engine(ex, budget=1000, slots=1, batching=b)
    ref[0] = eng
    eng.submit(Spec(0, geometry=0, R=3), 13)
    time.sleep(0.05)
    geos = [7, 7, 8, 7, 7, 7]
    for i, g in enumerate(geos, start=1):
        eng.submit(Spec(i, geometry=g, R=3), 13)
    assert eng.drain(timeout=30)
    eng.close()
    # FIFO head 1 takes 2 and 4 (R cap 9), then 3 alone (other geometry)... head 3 fails by injection
    assert ex.batches[0] == [0]
    assert ex.batches[1] == [1, 2, 4]
    assert ex.batches[2] == [3]
    assert ex.batches[3] == [5, 6]
    tk = {t.rid: t for t in eng.tickets}
    assert tk[1].batch == 3 and tk[1].result["batch"] == 3 and tk[3].error and tk[5].batch == 2
    assert eng.policy.used == 0
    st = latency_stats(eng.tickets)
    assert st["batched"] == 5


def test_request_footprint_of_a_batch():
    """A batch is one block solve over the stacked directions: below the sum of separate solves
    where the N-sized arrays dominate.  Not on small scenes, where the block Hessenberg matrix
    (R^2 m^2) can outweigh them, and not always above its largest request, whose pair sum may take
    the symmetric kernel with its per-distance slices where the batch takes the matrix cores."""
    for t_min, t_max, below_sum in ((4, 16, False), (300, 400, True)):
        specs = w.serving.request_stream(8, rate=1.0, seed=3, t_min=t_min, t_max=t_max, p_sweep=0.9)
        geo = specs[0].geometry
        same, R = [], 0
        for s in specs:  # a batch the engine could form: one geometry, at most 64 directions
            if s.geometry == geo and R + s.scene.R <= 64:
                same.append(s)
                R += s.scene.R
        assert len(same) >= 2
        joint = request_footprint(same)
        assert joint > 0
        if below_sum:
            assert joint < sum(request_footprint([s]) for s in same)


def test_footprint_follows_the_symmetric_slice_budget():
    """The symmetric pair kernel's partial slices, as the footprint counts them: 2000 bodies of 128
    points in 2D (the starfish layout) keep one slice per group distance (562 slices of N complex64
    values) under the default budget, and 128 (64 offset chunks, 64 source-side) when a one-byte
    budget asks for the shape whose 8 waves share each source tile."""
    from paper_2603_19113_amd import mfs

    shape_of = np.zeros(2000, dtype=np.int32)
    ks = [128]
    N = 2000 * 128
    before = mfs.sym_slice_budget(0)
    try:
        one_wave = mfs.solve_footprint(2, shape_of, ks, 1, 2000, basis32=True)
        mfs.sym_slice_budget(1)
        shared = mfs.solve_footprint(2, shape_of, ks, 1, 2000, basis32=True)
    finally:
        mfs.sym_slice_budget(before if before != 4 << 30 else 0)
    expected = (562 - 128) * N * 8
    assert 0.98 * expected <= one_wave - shared <= 1.02 * expected, (one_wave - shared, expected)
