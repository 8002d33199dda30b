"""Host logic of bench.py on the CPU: the one-GPU guard, the roofline flop counts and the lookup of
the committed traffic record (which must match workload, kernel, launch shape and kernel source)."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_flop_counts_per_pair():
    # plain kernel, one right-hand side: phi (34 in 2D, 26 in 3D) + one complex multiply-add (8)
    assert bench.flop_per_pair_plain(2, 1) == 42 and bench.flop_per_pair_plain(3, 1) == 34
    # symmetric kernel: phi once per unordered pair, two multiply-adds: (34 + 16) / 2
    assert bench.flop_per_pair_sym(2, 1) == 25 and bench.flop_per_pair_sym(3, 1) == 21
    # phi shared by R right-hand sides
    assert bench.flop_per_pair_plain(2, 4) == 34 / 4 + 8
    assert bench.flop_per_pair_sym(2, 4) == (34 / 4 + 16) / 2


def test_traffic_record_lookup():
    name = "ghat_sym_kernel<2> (G_hat, FP32, symmetric)"
    got = bench.stored_traffic("starfish2000", "starfish2000_kappa10", name, 63)
    assert got is not None and got > 1e9  # the committed record matches the current kernel source
    assert bench.stored_traffic("starfish2000", "starfish2000_kappa10", name, 126) is None  # other launch shape
    assert bench.stored_traffic("starfish2000", "starfish500_kappa10", name, 63) is None     # other scene
    assert bench.stored_traffic("disks16", "disks16_kappa5", name, 63) is None              # no record
    assert bench.stored_traffic("starfish2000", "starfish2000_kappa10",
                                "ghat_bodyphase_kernel<2,2,1> (G_hat, FP32)", 63) is None


def test_default_workload_is_the_largest_single_gpu_scene():
    import workloads as w

    ap_default = None
    src = open(os.path.join(ROOT, "bench.py")).read()
    for line in src.splitlines():
        if 'add_argument("--workload", default=' in line:
            ap_default = line.split('default="')[1].split('"')[0]
    assert ap_default == "spheres1000"
    pairs = {k: w.make_scene(k).n_pairs() for k in ("starfish2000", "spheres1000")}
    assert pairs["spheres1000"] > pairs["starfish2000"]
    assert set(bench.DEFAULT_RESTART) == set(w.CONFIGS)
