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


def test_traffic_record_lookup(tmp_path):
    """A counter record is used only for its workload's scene, kernel, launch shape and the kernel
    source it was taken with (anything else gives traffic = null)."""
    name = "ghat_sym16_kernel<1> (G_hat, FP32, symmetric, 16-point sub-blocks)"
    rec = tmp_path / "ghat_f32_spheres1000_traffic.md"
    rec.write_text("# record\nscene: spheres1000_kappa3\nkernel: ghat_sym16_kernel<1>\nnchunks: 37\n"
                   f"traffic_bytes_per_launch: 123456789\nkernel_source_sha256: {bench.kernel_source_sha256(name)}\n")
    got = bench.stored_traffic("spheres1000", "spheres1000_kappa3", name, 37, folder=str(tmp_path))
    assert got == 123456789
    assert bench.stored_traffic("spheres1000", "spheres1000_kappa3", name, 38, folder=str(tmp_path)) is None
    assert bench.stored_traffic("spheres1000", "spheres500_kappa3", name, 37, folder=str(tmp_path)) is None
    assert bench.stored_traffic("spheres1000", "spheres1000_kappa3", "ghat_sym_kernel<3,1> (G_hat)", 37,
                                folder=str(tmp_path)) is None
    assert bench.stored_traffic("disks16", "disks16_kappa5", name, 37, folder=str(tmp_path)) is None
    rec.write_text(rec.read_text().replace(bench.kernel_source_sha256(name), "0" * 64))  # kernel changed since
    assert bench.stored_traffic("spheres1000", "spheres1000_kappa3", name, 37, folder=str(tmp_path)) is None


def test_traffic_hash_follows_the_kernel_source():
    """The matrix-core kernels and the vector-unit kernels live in different files: a change to one
    leaves the other's counter records valid."""
    mc = bench.kernel_source_sha256("ghat_mfma16_kernel<2> (G_hat, FP16 matrix cores, split operands)")
    assert mc == bench.kernel_source_sha256("ghat_mfma_kernel<2> (G_hat, FP32 matrix cores)")
    assert mc != bench.kernel_source_sha256("ghat_sym16_kernel<1> (G_hat, FP32, symmetric, 16-point sub-blocks)")


def test_roofline_uses_the_algorithmic_work_per_pair():
    # phi and one complex multiply-add per pair: 45 flop-equivalents in 2D, 25 in 3D
    assert bench.alg_flop_per_pair(2, 1) == 45 and bench.alg_flop_per_pair(3, 1) == 25
    assert bench.alg_flop_per_pair(3, 4) == 17 / 4 + 8
    assert bench.PEAK_FP32_VECTOR_TFLOPS == 157.3


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
