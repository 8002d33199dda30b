"""Benchmark of the multibody MFS scattering hot path on one MI355X.

One step = one pass of the whole path over one synthetic scene:
  build S for every shape on the GPU (FP64 least squares)      -> mfs_build_S
  pack the scene (equivalent points, body tables)              -> mfs_scene_create
  plane-wave Dirichlet data at the equivalent points           -> mfs_plane_wave
  solve (I + S G_hat) q = S v to 1e-8 relative residual with FP32 pair sums and S products inside
  FP64 GMRES and FP64 iterative refinement                     -> mfs_solve (MFS_MIXED)
  scattered field at far targets                               -> mfs_eval_field
Default workload: 1000 unit spheres in 3D, kappa 3, 400 equivalent points each (N = 400,000,
1.598e11 off-body pairs per operator application): the largest single-GPU scene by pair evaluations
per matvec.  `--workload starfish2000` runs the 2000-starfish scene (one step takes minutes there:
the system needs ~6 GMRES iterations per body).

Prints one JSON line.  value = Helmholtz pair evaluations performed in the timed steps divided by
their wall time (whole-job throughput; the geometry is generated before timing starts).
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Helmholtz pair-evals/s per matvec; GMRES solve time @1e-8 rel res; p50/p99"
# Algorithmic work of one off-body pair (phi and one complex multiply-add), in flop-equivalents
# (FMA = 2, transcendental = 1), counted on the far-field branch of a plain FP32 evaluation:
# 2D ~27 VALU operations and 4-5 transcendentals = 45, 3D ~15 VALU and 3 transcendentals = 25.
# The roofline's `achieved` is this work per launch divided by the launch time, whatever the kernel
# does to get there (the symmetric kernels evaluate phi once per unordered pair, so they do less).
ALG_FLOP_PER_PAIR = {2: 45, 3: 25}
ALG_PHI_FLOP = {d: f - 8 for d, f in ALG_FLOP_PER_PAIR.items()}  # phi alone, without the 8-flop complex MAC


def alg_flop_per_pair(dim: int, R: int) -> float:
    """Algorithmic work per pair and right-hand side: phi shared by the R right-hand sides, one
    complex multiply-add each."""
    return ALG_PHI_FLOP[dim] / R + 8


# What the FP32 kernels themselves execute per pair (FMA = 2, transcendental = 1), counted on their
# far branch.  2D: u = sum_d dl_d (dl_d + 2 dc_d) (8), r^2 (1), rsq (1), r (1), D + r (1), rcp (1),
# delta (1), 1/r^2 (1), modulus poly (4), phase poly (5), phase sum (3), fract (1), sqrt (1),
# amplitude (1), sin + cos (2), (re, im) (2), complex multiply-add (8) = 42.
# 3D: u (12), r^2, rsq, r, D + r, rcp, delta (6), phase fma (2), fract (1), 1/(4 pi r) (1),
# sin + cos (2), (re, im) (2), complex multiply-add (8) = 34.
FLOP_PER_PAIR_F32 = {2: 42, 3: 34}
# phi alone, without the complex multiply-add (8): 34 and 26.
PHI_FLOP_F32 = {d: f - 8 for d, f in FLOP_PER_PAIR_F32.items()}


def flop_per_pair_plain(dim: int, R: int) -> float:
    """Plain kernels: phi once per (ordered) pair, shared by the R right-hand sides of a launch."""
    return PHI_FLOP_F32[dim] / R + 8


def flop_per_pair_sym(dim: int, R: int) -> float:
    """Symmetric kernel: phi once per unordered pair and two complex multiply-adds per right-hand
    side, i.e. (phi / R + 16) / 2 per ordered pair and right-hand side (R = 1: 25 in 2D, 21 in 3D)."""
    return (PHI_FLOP_F32[dim] / R + 16) / 2


# MI355X FP32 vector peak, 157.3 TFLOP/s (256 CUs x 4 SIMDs x 2.4 GHz x 64 flop per cycle with the
# packed two-wide FP32 instructions).  Every HIP build here disables packed FP32, so these kernels
# issue one-wide FP32 at most: 78.6 TFLOP/s, reported beside it.
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
# Many right-hand sides: G_hat tile x charge block on the FP32 matrix cores (dense FP32 MFMA peak).
FLOP_PER_PAIR_RHS_MFMA = 8
PEAK_FP32_MFMA_TFLOPS = 157.3
# The same contraction as FP16 products of split operands (hi + lo, three products per real product):
# 3 x 8 = 24 FP16 flop per (pair, right-hand side), against the dense FP16 matrix-core peak.
FLOP_PER_PAIR_RHS_SPLIT16 = 24
PEAK_FP16_MFMA_TFLOPS = 2500.0


# Host threads one GPU's share of the benchmark host may use.
CPU_SHARE_PER_GPU = 16

# Krylov basis length per workload: room for the whole solve without restarts (restarts stall these
# systems, and a deflated correction solve needs its vectors after the kept ones).
DEFAULT_RESTART = {"starfish2000": 16000, "spheres1000": 2000, "mixed2000_R64": 1000, "disks16": 400}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha256(kernel_name: str = "") -> str:
    """Hash of the sources of a pair kernel (the matrix-core kernels' file or the vector-unit kernels'
    file, with the headers both share), recorded with every traffic measurement."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2603_19113_amd", "csrc")
    main = "mc_kernels.hip" if kernel_name.startswith("ghat_mfma") else "pair_kernels.hip"
    return hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                   for f in (main, "bodyphase.h", "phi.h"))).hexdigest()


def stored_traffic(key: str, scene_name: str, kernel_name: str, nchunks: int, folder: str | None = None):
    """HBM bytes per launch of the FP32 G_hat kernel from the committed rocprofv3 counter summary of
    this workload (profiles/ghat_f32_<key>_traffic.md), or None if there is none, or it is for another
    scene, kernel or launch shape, or the kernel source has changed since the counters were taken."""
    path = os.path.join(folder or os.path.join(ROOT, "profiles"), f"ghat_f32_{key}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha256", "nchunks",
                                                     "kernel", "scene"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if not fields.get("kernel") or not kernel_name.startswith(fields["kernel"]):
        return None
    if fields.get("scene", scene_name) != scene_name:
        return None
    if fields.get("kernel_source_sha256") != kernel_source_sha256(kernel_name) or "traffic_bytes_per_launch" not in fields:
        return None
    if fields.get("nchunks") != str(nchunks):
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(sc, seconds: float) -> dict:
    """Time the FP64 oracle's G_hat rows (thread pool over row blocks) on a bounded row sample."""
    import numpy as np

    from oracle import global_system as gs

    xh, ptr, bo = gs.pack(sc)
    try:
        host_cores = len(os.sched_getaffinity(0))
    except AttributeError:
        host_cores = os.cpu_count() or 1
    # the oracle's thread pool takes every core of the affinity mask, up to the 16-thread CPU share
    # that one GPU gets on the benchmark hosts (both counts are reported)
    cores = max(1, min(host_cores, CPU_SHARE_PER_GPU))
    rng = np.random.default_rng(5)
    q = rng.standard_normal((1, sc.N)) + 1j * rng.standard_normal((1, sc.N))
    order = rng.permutation(sc.N)
    done, pairs, t_used = 0, 0.0, 0.0
    batch = max(cores * 8, 64)
    while t_used < seconds and done < sc.N:
        rows = np.sort(order[done:done + batch])
        t0 = time.perf_counter()
        gs.ghat_apply(xh, bo, sc.kappa, q, rows=rows, workers=cores, block=8)
        t_used += time.perf_counter() - t0
        k_rows = (ptr[bo[rows] + 1] - ptr[bo[rows]]).astype(np.float64)
        pairs += float(np.sum(sc.N - k_rows))
        done += rows.size
    return {"value": pairs / t_used, "unit": "pair-evals/s", "cores": cores, "host_cores": host_cores,
            "kind": "oracle",
            "sample": f"{done} of {sc.N} G_hat rows x all {sc.N} sources (FP64 scipy Hankel, "
                      f"{pairs:.3e} pairs in {t_used:.1f} s)"}


def serve(args, w, torch) -> int:
    """Poisson request stream through the serving engine: continuous admission by HBM footprint,
    per-slot streams, batching of requests on one geometry, cached device memory.

    The arrival rate is 0.7 x the sustained capacity measured on a calibration burst drawn from the
    same generator (another seed), unless --rate is given."""
    from paper_2603_19113_amd import mfs
    from paper_2603_19113_amd.serve import Engine, GpuExecutor, latency_stats, replay, request_batching, \
        request_footprint

    gen = dict(t_min=args.serve_tmin, t_max=args.serve_tmax, p_sweep=args.p_sweep)
    specs = w.serving.request_stream(args.serve, rate=1.0, seed=20260318, **gen)
    cal = w.serving.request_stream(max(8, args.serve // 4), rate=1.0, seed=20260319, **gen)
    budget = int(0.8 * torch.cuda.get_device_properties(0).total_memory)
    ex = GpuExecutor(args.slots, tol=args.tol, keep_solution=False)
    for s in cal + specs:  # the S library: one FP64 build per (shape, wavenumber), untimed
        for key, sh in zip(s.shape_keys, s.scene.shapes):
            ex.S(s.scene.dim, key, sh, s.scene.kappa, ex.streams[0])
    torch.cuda.synchronize()
    batching = None if args.no_batching else request_batching()

    def done(t):
        info = t.result["info"] if t.result else {}
        log(f"[serve] request {t.rid} {'failed' if t.error else 'done'}: {t.finish - t.arrival:.2f} s "
            f"(batch {t.batch}, relres {info.get('relres_max', float('nan')):.1e})")

    def run(stream, time_scale):
        eng = Engine(ex, budget=budget, slots=args.slots, batching=batching, on_done=done)
        t0 = time.perf_counter()
        tickets = replay(eng, stream, [request_footprint([s]) for s in stream], time_scale=time_scale)
        wall = time.perf_counter() - t0
        eng.close()
        return tickets, wall

    rate = args.rate
    capacity = None
    if rate <= 0.0:
        tk, wall = run(cal, 0.0)  # burst: every calibration request queued at once
        capacity = len(cal) / wall
        rate = 0.7 * capacity
        print(f"[serve] calibration: {len(cal)} requests in {wall:.2f} s -> capacity {capacity:.2f}/s, "
              f"rate {rate:.2f}/s", file=sys.stderr, flush=True)
    pool0 = mfs.pool_stats()
    tickets, wall = run(specs, 1.0 / rate)
    pool1 = mfs.pool_stats()
    st = latency_stats(tickets)
    fails = [t.error for t in tickets if t.error]
    worst = max((t.result["info"]["relres_max"] for t in tickets if not t.error), default=float("nan"))
    out = {"metric": "serving: p50/p99 latency and solves/s", "n_requests": len(specs), "rate_per_s": rate,
           "capacity_per_s": capacity, "slots": args.slots, "batching": batching is not None,
           "hbm_budget_bytes": budget, "wall_s": wall, **st, "relres_max": worst, "errors": fails[:3],
           "tol": args.tol, "pool_hits": pool1["hits"] - pool0["hits"], "pool_misses": pool1["misses"] - pool0["misses"],
           "requests": f"2D (disk, ellipse, starfish, kite, teardrop, C-shape, rod; kappa 5/10/20) and 3D (sphere, "
                       f"ellipsoid, torus; kappa 3/5), "
                       f"{args.serve_tmin}..{args.serve_tmax} bodies log-uniform, 1..16 directions, "
                       f"{args.p_sweep:g} of requests revisit an earlier geometry"}
    print(json.dumps(out), flush=True)
    return 0


def near(args, sc, mfs, torch, np) -> int:
    """Reconstruction of every body's MFS sources and field evaluation near the bodies (Sec. 4.6) on the
    benchmark scene, timed with HIP events.  The equivalent sources are seeded random numbers: the work
    does not depend on their values, and a full solve is not needed to time these steps."""
    built = [mfs.build_S(s, sc.kappa) for s in sc.shapes]
    recons = [mfs.Recon(s, sc.kappa) for s in sc.shapes]
    scene = mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                      [b.S64 for b in built], [b.S32 for b in built])
    R = 1
    mt, nt = mfs.near_sizes(scene, recons)
    v = torch.empty((R, mt), dtype=torch.complex128, device="cuda")
    mfs.plane_wave_colloc(scene, recons, sc.directions[:R], v)
    g = torch.Generator(device="cuda").manual_seed(20260318)
    qhat = torch.complex(torch.randn((R, scene.N), generator=g, device="cuda", dtype=torch.float64),
                         torch.randn((R, scene.N), generator=g, device="cuda", dtype=torch.float64))
    qm = torch.empty((R, nt), dtype=torch.complex128, device="cuda")
    # targets: 32 per body, on a circle (sphere: Fibonacci) between the body and its proxy surface
    per = 32
    tpl = []
    for s in sc.shapes:
        rad = 0.5 * (s.bounding_radius + s.proxy_radius)
        tpl.append(w_points(sc.dim, per, rad))
    tg_h = np.concatenate([tpl[int(sh)] + sc.centres[t][None, :] for t, sh in enumerate(sc.shape_of)], 0)
    tg = torch.from_numpy(tg_h).cuda()
    u = torch.empty((R, tg_h.shape[0]), dtype=torch.complex128, device="cuda")
    st = torch.cuda.current_stream()

    def timed(fn, reps=3):
        fn()  # warm-up (first call builds the scene's near-field tables)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    t_rec = timed(lambda: mfs.reconstruct(scene, recons, v, qhat, qm))
    t_eval = timed(lambda: mfs.eval_field_near(scene, recons, qhat, qm, tg, u))
    # pair count of the near evaluation: per target, n of each body whose proxy surface holds it, k of the others
    k_of = np.array([s.eqpts.shape[0] for s in sc.shapes])[sc.shape_of]
    n_of = np.array([s.src.shape[0] for s in sc.shapes])[sc.shape_of]
    psi = np.array([s.proxy_radius for s in sc.shapes])[sc.shape_of]
    pairs = 0.0
    for i0 in range(0, tg_h.shape[0], 4096):
        blk = tg_h[i0:i0 + 4096]
        inside = np.linalg.norm(blk[:, None, :] - sc.centres[None, :, :], axis=2) < psi[None, :]
        pairs += float(np.sum(np.where(inside, n_of[None, :], k_of[None, :])))
    out = {"workload": sc.name, "N": scene.N, "T": sc.T, "R": R, "mode": "reconstruction and near field",
           "reconstruct_ms": t_rec, "near_targets": int(tg_h.shape[0]), "eval_near_ms": t_eval,
           "eval_near_pairs": pairs, "eval_near_pair_evals_per_s_fp64": pairs / (t_eval * 1e-3),
           "data": "seeded random equivalent sources (timing only)"}
    for r in recons:
        r.close()
    scene.close()
    print(json.dumps(out), flush=True)
    return 0


def w_points(dim, count, radius):
    import workloads as w

    return w.circle_points(count, radius, 0.1) if dim == 2 else w.fibonacci_sphere(count, radius)


def compare(args, sc, mfs, torch, np) -> int:
    """Mixed-precision batched solve vs plain FP64 GMRES, one right-hand side at a time."""
    built = [mfs.build_S(s, sc.kappa) for s in sc.shapes]
    scene = mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                      [b.S64 for b in built], [b.S32 for b in built])
    R = sc.R
    v = torch.empty((R, scene.N), dtype=torch.complex128, device="cuda")
    mfs.plane_wave(scene, sc.directions, v)
    q_mixed = torch.empty_like(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    use_block = R > 1 and not args.no_block
    info_m = mfs.solve(scene, v, q_mixed, tol=args.tol, maxit=60000, restart=args.restart, max_refine=20,
                       inner_tol=args.inner_tol, prec=mfs.MFS_MIXED, verbose=min(args.verbose, 1),
                       basis32=not args.basis64, deflate=not args.no_deflate, block=use_block)
    t_mixed = time.perf_counter() - t0
    log(f"[compare] mixed, {R} RHS together: {t_mixed:.2f} s  {info_m}")
    q64 = torch.empty_like(v)
    t_fp64, it64, rel64 = 0.0, 0, 0.0
    n64 = R if args.fp64_rhs <= 0 else min(R, args.fp64_rhs)
    for r in range(n64):
        vr = v[r:r + 1].contiguous()
        qr = torch.empty_like(vr)
        t0 = time.perf_counter()
        info = mfs.solve(scene, vr, qr, tol=args.tol, maxit=60000, restart=args.restart, prec=mfs.MFS_FP64,
                         verbose=0)
        t_fp64 += time.perf_counter() - t0
        it64 += info["n_matvec64"]
        rel64 = max(rel64, info["relres_max"])
        q64[r].copy_(qr[0])
        log(f"[compare] fp64 rhs {r}: {info['t_total_s']:.2f} s  {info['n_matvec64']} FP64 operator applications")
    diff = float(torch.linalg.norm(q_mixed[:n64] - q64[:n64]) / torch.linalg.norm(q64[:n64]))
    # with --fp64-rhs K < R only K single-RHS solves run; their mean time stands for the other R - K
    t_fp64_all = t_fp64 * R / n64
    out = {"workload": sc.name, "N": scene.N, "T": sc.T, "R": R, "tol": args.tol, "restart": args.restart,
           "mixed_batched": {"seconds": t_mixed, "relres_max": info_m["relres_max"],
                             "krylov": "block GMRES" if use_block else "GMRES per column",
                             "fp32_operator_applications": info_m["n_matvec32"],
                             "fp64_operator_applications": info_m["n_matvec64"]},
           "fp64_single_rhs": {"seconds": t_fp64_all, "timed_rhs": n64, "extrapolated": n64 < R,
                               "relres_max": rel64, "fp64_operator_applications": it64},
           "speedup": t_fp64_all / t_mixed, "solution_rel_diff": diff}
    print(json.dumps(out), flush=True)
    scene.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="spheres1000",
                    choices=["starfish2000", "spheres1000", "mixed2000_R64", "disks16"])
    ap.add_argument("--bodies", type=int, default=None, help="override T (scaled scene, same density)")
    ap.add_argument("--restart", type=int, default=0,
                    help="Krylov basis size (0: the workload's default, which keeps the whole basis resident)")
    ap.add_argument("--inner-tol", type=float, default=3e-6,
                    help="first inner solve stops here: below ~7e-6 the FP32 operator error caps the true residual")
    ap.add_argument("--basis64", action="store_true",
                    help="keep the Krylov basis of the mixed solve in complex128 (default: complex64)")
    ap.add_argument("--matvecs", type=int, default=0,
                    help="profiling mode: replace the solve by this many mixed operator applications")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="profiling: first copy a buffer of this many MiB (calibrates rocprof byte counters)")
    ap.add_argument("--sym-slice-budget", type=int, default=0, metavar="BYTES",
                    help="slice budget of the symmetric pair kernel (0: the library default); 1 forces the "
                         "form whose 8 waves share each source tile")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--mc-fp32", action="store_true",
                    help="many right-hand sides: FP32 matrix-core products instead of FP16 products of "
                         "split operands")
    ap.add_argument("--no-block", action="store_true",
                    help="several right-hand sides: one Krylov space per column instead of block GMRES")
    ap.add_argument("--no-deflate", action="store_true",
                    help="correction solves restart from scratch instead of deflating the first inner "
                         "solve's Krylov space")
    ap.add_argument("--rhs", type=int, default=0,
                    help="use only the first RHS incident directions of the workload (0: all of them)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner (run before the warm-up, outside the timed steps)")
    ap.add_argument("--launch-shape", default=None, metavar="NCHUNKS:RT[:SYM]",
                    help="use this pair-sum launch shape on every scene instead of tuning (profiling runs); "
                         "SYM 1 = symmetric kernel where it applies, 0 = plain kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--verbose", type=int, default=2, help="solver progress lines on stderr")
    ap.add_argument("--serve", type=int, default=0,
                    help="instead of the benchmark line: replay this many Poisson-arriving requests through "
                         "the serving engine and report p50/p99 latency and solves/s")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="--serve: mean arrivals per second (0: 0.7 x capacity from a calibration burst)")
    ap.add_argument("--slots", type=int, default=4, help="--serve: concurrent requests")
    ap.add_argument("--serve-tmin", type=int, default=8, help="--serve: fewest bodies per request")
    ap.add_argument("--serve-tmax", type=int, default=128, help="--serve: most bodies per request")
    ap.add_argument("--p-sweep", type=float, default=0.3,
                    help="--serve: share of requests that revisit an earlier geometry with new directions")
    ap.add_argument("--no-batching", action="store_true", help="--serve: one solve per request")
    ap.add_argument("--near", action="store_true",
                    help="instead of the benchmark line: time the reconstruction of the MFS sources and the "
                         "near-body field evaluation (seeded equivalent sources)")
    ap.add_argument("--fp64-rhs", type=int, default=0,
                    help="--compare: time only this many single-RHS FP64 solves and scale to R (0: all)")
    ap.add_argument("--compare", action="store_true",
                    help="instead of the benchmark line: time the mixed-precision (batched) solve against the "
                         "plain FP64 single-RHS form (each right-hand side solved alone) on the same scene")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is a "
              f"design note, not an implemented path.", file=sys.stderr)
        return 2

    if args.restart <= 0:
        args.restart = DEFAULT_RESTART[args.workload]

    import numpy as np
    import torch

    import workloads as w
    from paper_2603_19113_amd import mfs

    mfs.load()
    torch.cuda.set_device(0)
    mfs.sym_slice_budget(args.sym_slice_budget)
    if args.serve > 0:
        return serve(args, w, torch)
    sc = w.make_scene(args.workload, T=args.bodies)
    if args.rhs:
        if not 1 <= args.rhs <= sc.R:
            print(f"--rhs must be in 1..{sc.R} for this workload", file=sys.stderr)
            return 2
        sc.directions = sc.directions[:args.rhs]
    R = sc.R
    dirs = sc.directions
    use_block = R > 1 and not args.no_block  # one block Krylov space for the R incident directions
    targets = torch.from_numpy(w.far_targets(sc, 256)).cuda()
    log(f"[bench] workload {sc.name}: T={sc.T} N={sc.N} R={R} pairs/matvec={sc.n_pairs():.4e}")
    if args.copy_mib > 0:
        # a plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # scale between counter units and bytes for the pair kernel's counters in the same run
        src = torch.empty(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    forced = None
    if args.launch_shape:
        parts = [int(x) for x in args.launch_shape.split(":")]
        forced = (parts[0], parts[1], parts[2] if len(parts) > 2 else -1)

    def build_all():
        return [mfs.build_S(s, sc.kappa) for s in sc.shapes]

    def make_scene(built=None):
        built = built or build_all()
        scene = mfs.Scene(sc.dim, sc.kappa, sc.shape_of, sc.centres, [s.eqpts for s in sc.shapes],
                          [b.S64 for b in built], [b.S32 for b in built])
        if forced:
            mfs.tune_set(scene, R, mfs.MFS_MIXED, *forced)
        if args.mc_fp32 and mfs.pair_kernel(scene, R, mfs.MFS_MIXED) == mfs.MFS_PAIR_MC_F16X3:
            mfs.set_split_fp16(scene, False)
        return scene

    def step():
        """One pass of the whole path; returns the solver's info with the wall time of each phase."""
        t0 = time.perf_counter()
        built = build_all()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        scene = make_scene(built)
        v = torch.empty((R, scene.N), dtype=torch.complex128, device="cuda")
        mfs.plane_wave(scene, dirs, v)
        q = torch.empty_like(v)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if args.matvecs > 0:
            # profiling mode: the operator applications of a solve without the Krylov recurrence
            q32 = v.to(torch.complex64)
            y32 = torch.empty_like(q32)
            for _ in range(args.matvecs):
                mfs.apply(scene, q32, y32, mfs.MFS_FP32)
                q32, y32 = y32, q32
            q.copy_(q32)
            info = {"relres_max": float("nan"), "n_matvec32": args.matvecs, "n_matvec64": 0, "n_refine": 0,
                    "t_total_s": 0.0, "n_reorth": 0, "status": "profile"}
        else:
            info = mfs.solve(scene, v, q, tol=args.tol, maxit=60000, restart=args.restart, max_refine=20,
                             inner_tol=args.inner_tol, prec=mfs.MFS_MIXED, verbose=args.verbose,
                             basis32=not args.basis64, deflate=not args.no_deflate, block=use_block)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        u = torch.empty((R, targets.shape[0]), dtype=torch.complex128, device="cuda")
        mfs.eval_field(scene, q, targets, u, mfs.MFS_FP64)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        scene.close()
        info["phase_s"] = {"build_S": t1 - t0, "scene_and_rhs": t2 - t1, "solve": t3 - t2, "field": t4 - t3}
        return info

    if args.compare:
        return compare(args, sc, mfs, torch, np)
    if args.near:
        return near(args, sc, mfs, torch, np)

    # launch shape of the FP32 pair sum: tuned once on this scene (the process-wide table then serves
    # the scenes the steps build), or the heuristic with --no-tune
    probe = make_scene()
    tune = None
    if not args.no_tune and not forced:
        t0 = time.perf_counter()
        tune = mfs.autotune(probe, R=R, prec=mfs.MFS_MIXED, reps=2)
        log(f"[bench] autotune ({time.perf_counter() - t0:.1f} s): {tune}")
    shape = mfs.tune_get(probe, R, mfs.MFS_MIXED)
    pair_kind = mfs.pair_kernel(probe, R, mfs.MFS_MIXED)
    probe.close()

    for i in range(args.warmup):
        t0 = time.perf_counter()
        info = step()
        log(f"[bench] warmup {i}: {time.perf_counter() - t0:.2f} s  {info}")

    mfs.timing_enable(True)
    times, infos = [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(info)
        ph = info["phase_s"]
        log(f"[bench] step {i}: {times[-1]:.2f} s  relres {info['relres_max']:.2e}  "
            f"matvec32 {info['n_matvec32']} matvec64 {info['n_matvec64']} refine {info['n_refine']}  "
            f"(S {ph['build_S']:.2f} s, scene {ph['scene_and_rhs']:.2f} s, solve {ph['solve']:.2f} s, "
            f"field {ph['field']:.3f} s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    ms32, n32, p32 = mfs.timing_read(mfs.MFS_KERNEL_PAIR_F32)
    ms64, n64, p64 = mfs.timing_read(mfs.MFS_KERNEL_PAIR_F64)
    mfs.timing_enable(False)

    shared = pair_kind in (mfs.MFS_PAIR_F32_SYM_SHARED, mfs.MFS_PAIR_F32_SYM16_SHARED)
    on_sym = shared or pair_kind in (mfs.MFS_PAIR_F32_SYM, mfs.MFS_PAIR_F32_SYM16)
    on_mfma = pair_kind in (mfs.MFS_PAIR_MC_F32, mfs.MFS_PAIR_MC_F16X3)
    split16 = pair_kind == mfs.MFS_PAIR_MC_F16X3
    sub_blocks = pair_kind in (mfs.MFS_PAIR_F32_SYM16, mfs.MFS_PAIR_F32_SYM16_SHARED)
    rt = shape["rhs_per_thread"] or (1 if R == 1 else 2 if R == 2 else 4)
    if sub_blocks:
        kernel_name = ("ghat_sym16_shared_kernel<%d,8> (G_hat, FP32, symmetric, 16-point sub-blocks, shared source tiles)"
                       % rt if shared else "ghat_sym16_kernel<%d> (G_hat, FP32, symmetric, 16-point sub-blocks)" % rt)
    elif on_sym:
        kernel_name = ("ghat_sym_shared_kernel<%d,%d,8> (G_hat, FP32, symmetric, shared source tiles)" % (sc.dim, rt)
                       if shared else "ghat_sym_kernel<%d,%d> (G_hat, FP32, symmetric)" % (sc.dim, rt))
    elif split16:
        kernel_name = "ghat_mfma16_kernel<%d> (G_hat, FP16 matrix cores, split operands)" % sc.dim
    elif on_mfma:
        kernel_name = "ghat_mfma_kernel<%d> (G_hat, FP32 matrix cores)" % sc.dim
    else:
        kernel_name = "ghat_bodyphase_kernel<%d,2,%d> (G_hat, FP32)" % (sc.dim, shape["rhs_per_thread"])
    traffic = stored_traffic(args.workload, sc.name, kernel_name, shape["nchunks"])
    total_pairs = p32 + p64
    value = total_pairs / wall
    avg32 = ms32 / max(n32, 1)
    pairs_per_launch32 = p32 / max(n32, 1)   # pair evaluations times right-hand sides
    rate = pairs_per_launch32 / (avg32 * 1e-3) if n32 else 0.0  # (pair, right-hand side) per second
    if split16:
        # the contraction as FP16 products of split operands: 24 FP16 flop per (pair, right-hand side)
        # (three products per real product of the 8-flop complex multiply-add), against the FP16
        # matrix-core peak; the FP32-equivalent rate (8 flop) is reported beside it
        alg_pp, kern_pp, bound, peak = FLOP_PER_PAIR_RHS_SPLIT16, FLOP_PER_PAIR_RHS_SPLIT16, "mfma", PEAK_FP16_MFMA_TFLOPS
    elif on_mfma:
        # the contraction on the FP32 matrix cores: 8 flop per (pair, right-hand side) complex multiply-add
        alg_pp, kern_pp, bound, peak = FLOP_PER_PAIR_RHS_MFMA, FLOP_PER_PAIR_RHS_MFMA, "mfma", PEAK_FP32_MFMA_TFLOPS
    else:
        alg_pp = alg_flop_per_pair(sc.dim, R)
        kern_pp = flop_per_pair_sym(sc.dim, R) if on_sym else flop_per_pair_plain(sc.dim, R)
        if on_sym and sub_blocks:
            kern_pp -= 1.0 / R  # no 1/(4 pi r) product and no fract per unordered pair: 2 flop less
        bound, peak = "alu", PEAK_FP32_VECTOR_TFLOPS
    achieved = alg_pp * rate / 1e12
    kernel_tflops = kern_pp * rate / 1e12
    solve_times = [i["t_total_s"] for i in infos]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair sums + f64 Krylov/refinement",
        "data": "synthetic (seeded geometry, no dataset)",
        "config": {"workload": sc.name, "T": sc.T, "N": sc.N, "R": R, "kappa": sc.kappa, "tol": args.tol,
                   "precision": "mixed", "restart": args.restart, "inner_tol": args.inner_tol,
                   "krylov_basis": "c128" if args.basis64 else "c64",
                   "krylov": "block GMRES (one space for the R directions)" if use_block else "GMRES per column"},
        "solve_s_p50": statistics.median(solve_times) if args.matvecs == 0 else None,
        "solve_s_p99": float(np.percentile(solve_times, 99)) if args.matvecs == 0 else None,
        "relres_max": max(i["relres_max"] for i in infos),
        "n_matvec32": infos[-1]["n_matvec32"],
        "n_matvec64": infos[-1]["n_matvec64"],
        "n_refine": infos[-1]["n_refine"],
        "n_reorth": infos[-1].get("n_reorth", 0),
        "phase_s_p50": {k: statistics.median(i["phase_s"][k] for i in infos) for k in infos[0]["phase_s"]},
        "mode": "profile (operator applications only)" if args.matvecs > 0 else "full solve",
        "pair_kernel_f32": {"launches": n32, "avg_ms": avg32, "rhs": R, "pairs_per_launch": pairs_per_launch32,
                            "pair_evals_per_s": pairs_per_launch32 / (avg32 * 1e-3) if n32 else 0.0},
        "launch_shape": {**shape, **({"tuned_ms": tune["ms"], "heuristic_ms": tune["ms_heuristic"],
                                      "tried": tune["n_tried"]} if tune else {})},
        "pair_kernel_f64": {"launches": n64, "avg_ms": ms64 / max(n64, 1),
                            "pair_evals_per_s": p64 / (ms64 * 1e-3) if n64 else 0.0},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": kernel_name, "avg_launch_ms": avg32,
                     ("alg_flop_per_pair" if not on_mfma else "alg_flop_per_pair_rhs"): alg_pp,
                     "kernel_flop_per_pair": kern_pp, "kernel_tflops": kernel_tflops,
                     **({"peak_unpacked_fp32": PEAK_FP32_UNPACKED_TFLOPS,
                         "kernel_frac_of_unpacked_peak": kernel_tflops / PEAK_FP32_UNPACKED_TFLOPS}
                        if not on_mfma else {}),
                     **({"fp32_equivalent_tflops": FLOP_PER_PAIR_RHS_MFMA * rate / 1e12,
                         "fp32_equivalent_frac_of_fp32_mfma_peak": FLOP_PER_PAIR_RHS_MFMA * rate / 1e12 / PEAK_FP32_MFMA_TFLOPS}
                        if split16 else {})},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a row sample ...")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
