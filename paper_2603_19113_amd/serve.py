"""Request loop for scattering solves on one GPU: continuous admission by HBM footprint.

Requests (scenes with one or more incident directions) arrive over time.  The engine keeps a FIFO
queue and a set of slots; the head of the queue is admitted as soon as a slot is free and its
estimated device footprint fits in the HBM budget next to the requests already running.  Each slot
runs its request on its own HIP stream (mixed-precision GMRES-IR through the C ABI, block GMRES for
several directions), so the work
of admitted requests overlaps on the device, and finished requests free their footprint for the
queue at once.  Scattering matrices are built once per (shape, wavenumber) and stay resident in a
shared library.  Results do not depend on what else runs: every kernel is deterministic and a
request's arithmetic never mixes with another's.

The admission policy and the slot/queue machinery are plain Python and take the executor as a
parameter, so they run on the CPU with a fake executor and a virtual clock.
"""

from __future__ import annotations

import collections
import queue as queue_mod
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable

import numpy as np


# ------------------------------------------------------------------ policy ---
def block_solve(R: int) -> bool:
    """Several right-hand sides (one request's directions, or a batch's) share one block Krylov
    space; the library's block solve takes up to 64."""
    return 2 <= R <= 64


def restart_for(T: int, kappa: float, dim: int, R: int = 1, cap: int = 4000, block_cap: int = 2000) -> int:
    """Krylov basis size, with room for the whole solve so that a request rarely restarts.  One
    right-hand side: GMRES needs about 6 steps per body at kappa = 10 in 2D (measured).  Block GMRES
    over R directions needs fewer block steps than one column needs steps, by a factor that grows
    with R: 17x at R = 64 on the 2000-body mixed scene (687 block steps against ~11,800); the basis
    is sized with R^0.6 (12x at 64, 3.5x at 8), which leaves room at small R, where restarted block
    cycles converge slowly (measured: 495 bodies, kappa 5, R = 8 stalls at 4e-7 after 30 cycles of
    125 block steps)."""
    est = int(8 * T * max(kappa, 3.0) / 10.0) + 200
    if block_solve(R):
        return max(64, min(block_cap, int(est / R ** 0.6)))
    return max(64, min(cap, est))


def footprint_bytes(dim: int, shape_of, k_of_shape, R: int, restart: int, n_targets: int = 0) -> int:
    """Device bytes a request holds while it runs: the library's own estimate for the scene and the
    solve (mfs_solve_footprint: tables, pair partial sums, Krylov workspace, solver vectors) plus the
    caller's vectors (v_hat and q_hat, complex128 R x N each, and the field at the targets)."""
    from . import mfs

    N = int(np.asarray(k_of_shape, np.int64)[np.asarray(shape_of)].sum())
    lib = mfs.solve_footprint(dim, shape_of, k_of_shape, R, restart, prec=mfs.MFS_MIXED, block=block_solve(R),
                              basis32=True, n_targets=n_targets)
    caller = 2 * R * N * 16 + R * max(n_targets, 1) * 16
    return int(lib + caller)


class Admission:
    """FIFO admission by footprint: the head enters when a slot is free and it fits the budget."""

    def __init__(self, budget: int, slots: int):
        self.budget = int(budget)
        self.slots = int(slots)
        self.used = 0
        self.running = 0
        self.peak_used = 0

    def fits(self, fp: int) -> bool:
        if fp > self.budget:
            raise ValueError(f"request needs {fp} bytes, more than the whole budget {self.budget}")
        return self.running < self.slots and self.used + fp <= self.budget

    def admit(self, fp: int):
        self.used += fp
        self.running += 1
        self.peak_used = max(self.peak_used, self.used)

    def release(self, fp: int):
        self.used -= fp
        self.running -= 1


# ------------------------------------------------------------------ engine ---
@dataclass
class Ticket:
    rid: int
    arrival: float
    footprint: int
    start: float = float("nan")
    finish: float = float("nan")
    batch: int = 1                      # requests that shared this request's solve
    admitted: int = -1                  # position in the admission order
    result: dict = field(default_factory=dict)
    error: str | None = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


@dataclass
class Batching:
    """Continuous batching across requests: queued requests with the same geometry key (same bodies
    and wavenumber, different incident fields) join the head of the queue in one multi-RHS solve."""
    key: Callable[[Any], Any]                  # spec -> hashable geometry key
    rhs: Callable[[Any], int]                  # spec -> right-hand sides it brings
    footprint: Callable[[list], int]           # specs of one batch -> device bytes of the joint solve
    max_rhs: int = 64


class Engine:
    """Slots x streams with one worker thread per slot and one dispatcher.

    executor(specs, slot) -> list of result dicts, one per spec, runs one batch on the slot."""

    def __init__(self, executor, budget: int, slots: int = 4, clock=time.monotonic, batching: Batching | None = None,
                 start: bool = True, on_done: Callable[[Ticket], None] | None = None):
        self.executor = executor
        self.on_done = on_done  # called from the worker for every finished ticket (progress, logging)
        self.policy = Admission(budget, slots)
        self.clock = clock
        self.batching = batching
        self.queue: collections.deque = collections.deque()
        self.lock = threading.Condition()
        self.free_slots = list(range(slots))
        self.inbox = [queue_mod.Queue() for _ in range(slots)]
        self.closed = False
        self.tickets: list[Ticket] = []
        self.n_admitted = 0
        self.workers = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(slots)]
        for t in self.workers:
            t.start()
        self.dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        if start:
            self.dispatcher.start()

    def start(self):
        """Start admitting (for an engine created with start=False, e.g. to queue a burst first)."""
        if not self.dispatcher.is_alive():
            self.dispatcher.start()

    def submit(self, spec, footprint: int, arrival: float | None = None) -> Ticket:
        t = Ticket(rid=spec.rid, arrival=self.clock() if arrival is None else arrival, footprint=footprint)
        with self.lock:
            if footprint > self.policy.budget:
                raise ValueError(f"request {spec.rid} needs {footprint} bytes, over the budget")
            self.queue.append((spec, t))
            self.tickets.append(t)
            self.lock.notify_all()
        return t

    def _take_batch(self):
        """Pop the head and, with batching on, every queued request on its geometry that still fits."""
        spec, t = self.queue.popleft()
        group = [(spec, t)]
        fp = t.footprint
        b = self.batching
        if b is not None:
            key = b.key(spec)
            nrhs = b.rhs(spec)
            for item in list(self.queue):
                s2 = item[0]
                if b.key(s2) != key or nrhs + b.rhs(s2) > b.max_rhs:
                    continue
                fp2 = b.footprint([x[0] for x in group] + [s2])
                if self.policy.used + fp2 > self.policy.budget:
                    continue
                group.append(item)
                self.queue.remove(item)
                nrhs += b.rhs(s2)
                fp = fp2
        return group, fp

    def _dispatch(self):
        while True:
            with self.lock:
                while not self.closed and not (self.queue and self.policy.fits(self.queue[0][1].footprint)):
                    self.lock.wait()
                if self.closed and not self.queue:
                    for box in self.inbox:
                        box.put(None)
                    return
                if not self.queue:
                    continue
                group, fp = self._take_batch()
                for _, t in group:
                    t.admitted = self.n_admitted
                    self.n_admitted += 1
                self.policy.admit(fp)
                slot = self.free_slots.pop()
            self.inbox[slot].put((group, fp))

    def _worker(self, slot: int):
        while True:
            job = self.inbox[slot].get()
            if job is None:
                return
            group, fp = job
            start = self.clock()
            for _, t in group:
                t.start = start
                t.batch = len(group)
            try:
                results = self.executor([s for s, _ in group], slot)
                for (_, t), res in zip(group, results):
                    t.result = res
            except Exception as e:  # a failed batch frees its slot; the error is reported on its tickets
                for _, t in group:
                    t.error = f"{type(e).__name__}: {e}"
            finish = self.clock()
            for _, t in group:
                t.finish = finish
            with self.lock:
                self.policy.release(fp)
                self.free_slots.append(slot)
                self.lock.notify_all()
            for _, t in group:
                t.done.set()
                if self.on_done is not None:
                    self.on_done(t)

    def drain(self, timeout: float | None = None) -> bool:
        deadline = None if timeout is None else time.monotonic() + timeout
        for t in list(self.tickets):
            left = None if deadline is None else max(0.0, deadline - time.monotonic())
            if not t.done.wait(left):
                return False
        return True

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        if self.dispatcher.is_alive():
            self.dispatcher.join(timeout=5.0)
        else:
            for box in self.inbox:
                box.put(None)
        for t in self.workers:
            t.join(timeout=5.0)


def latency_stats(tickets) -> dict:
    lat = np.array([t.latency for t in tickets if t.error is None])
    if lat.size == 0:
        return {"n": 0}
    first = min(t.arrival for t in tickets)
    last = max(t.finish for t in tickets)
    return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "solves_per_s": float(lat.size / max(last - first, 1e-9)),
            "failed": sum(1 for t in tickets if t.error is not None),
            "batched": sum(1 for t in tickets if t.batch > 1)}


# ------------------------------------------------------- request footprints ---
def request_footprint(specs) -> int:
    """Device bytes of one solve over the given requests (one geometry, their directions stacked)."""
    sc = specs[0].scene
    R = sum(s.scene.R for s in specs)
    return footprint_bytes(sc.dim, sc.shape_of, sc.k_of_shape, R, restart_for(sc.T, sc.kappa, sc.dim, R))


def request_batching(max_rhs: int = 64) -> Batching:
    """Requests on the same geometry (bodies, shapes, wavenumber) share one multi-RHS solve."""
    return Batching(key=lambda s: s.geometry, rhs=lambda s: s.scene.R, footprint=request_footprint, max_rhs=max_rhs)


# ------------------------------------------------------------- GPU executor ---
class GpuExecutor:
    """Runs one request through the C ABI on the slot's own stream.  S per (dim, shape, kappa) is
    built once (FP64, on the GPU) and shared by every request that uses that shape."""

    def __init__(self, slots: int, tol: float = 1e-8, inner_tol: float = 3e-6, keep_solution: bool = True):
        import torch

        from . import mfs

        self.mfs = mfs
        self.torch = torch
        mfs.load()
        self.streams = [torch.cuda.Stream() for _ in range(slots)]  # default priority
        self.library: dict = {}
        self.lib_lock = threading.Lock()
        self.tol = tol
        self.inner_tol = inner_tol
        self.keep_solution = keep_solution

    def S(self, dim, key, shape, kappa, stream):
        k = (dim, key, float(kappa))
        with self.lib_lock:
            if k not in self.library:
                self.library[k] = self.mfs.build_S(shape, kappa, stream=stream)
            return self.library[k]

    def __call__(self, specs, slot: int) -> list:
        """Solve a batch of requests on one geometry as one mixed-precision solve over their stacked
        incident directions (block GMRES with iterative refinement for 2..64 of them, GMRES-IR for
        one), then split the solution rows back per request."""
        torch, mfs = self.torch, self.mfs
        spec0 = specs[0]
        sc = spec0.scene
        if any(s.geometry != spec0.geometry for s in specs):
            raise ValueError("a batch must share one geometry")
        dirs = np.concatenate([np.atleast_2d(s.scene.directions) for s in specs], axis=0)
        st = self.streams[slot]
        with torch.cuda.stream(st):
            built = [self.S(sc.dim, key, sh, sc.kappa, st) for key, sh in zip(spec0.shape_keys, sc.shapes)]
            scene = mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                              [b.S64 for b in built], [b.S32 for b in built])
            try:
                R = dirs.shape[0]
                v = torch.empty((R, scene.N), dtype=torch.complex128, device="cuda")
                mfs.plane_wave(scene, dirs, v, stream=st)
                q = torch.empty_like(v)
                restart = restart_for(sc.T, sc.kappa, sc.dim, R)
                info = mfs.solve(scene, v, q, tol=self.tol, maxit=200000, restart=restart, max_refine=30,
                                 inner_tol=self.inner_tol, prec=mfs.MFS_MIXED, stream=st, basis32=True,
                                 deflate=True, block=block_solve(R))
                qh = q.cpu().numpy() if self.keep_solution else None  # synchronises the slot's stream
                st.synchronize()
                N = scene.N
            finally:
                scene.close()
        out, off = [], 0
        for s in specs:
            r = s.scene.R
            res = {"info": info, "N": N, "T": sc.T, "R": r, "batch_R": R, "dim": sc.dim, "kappa": sc.kappa,
                   "restart": restart}
            if qh is not None:
                res["qhat"] = qh[off:off + r]
            out.append(res)
            off += r
        return out


def replay(engine: Engine, specs, footprints, time_scale: float = 1.0):
    """Submit requests at their (scaled) arrival times, then wait for all of them."""
    t0 = time.monotonic()
    for spec, fp in zip(specs, footprints):
        delay = t0 + spec.arrival * time_scale - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        engine.submit(spec, fp)
    engine.drain()
    return engine.tickets
