"""The C ABI library on the CPU: it loads, exports every entry point include/mfs.h declares, and
rejects invalid arguments before touching the device (no compute calls here)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_19113_amd import mfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mfs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfs_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mfs.LIB_PATH):
        pytest.fail("libmfs.so is not built: run python -m paper_2603_19113_amd.build")
    return mfs.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("mfs_build_S", "mfs_apply", "mfs_solve", "mfs_eval_field", "mfs_scene_create"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(mfs.EXPORTS) == set(_declared_functions())


def test_static_scratch_size_matches_header():
    text = open(os.path.join(ROOT, "include", "mfs.h")).read()
    m = re.search(r"#define MFS_STATIC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == mfs.STATIC_SCRATCH_BYTES


def test_version_and_error_string(lib):
    assert lib.mfs_version() >= 100
    assert isinstance(lib.mfs_last_error(), bytes)


def test_invalid_arguments_rejected_without_device(lib):
    out = ctypes.c_void_p(0)
    k = np.array([4], np.int64)
    # dim 4 is rejected before any allocation
    assert lib.mfs_scene_create(4, 1.0, 1, None, None, None, 1, k.ctypes.data, None, None, None,
                                ctypes.byref(out)) == -1
    assert b"dim" in lib.mfs_last_error()
    # non-positive wavenumber
    assert lib.mfs_scene_create(2, -1.0, 1, None, None, None, 1, k.ctypes.data, None, None, None,
                                ctypes.byref(out)) == -1
    # null scene for every scene entry point
    assert lib.mfs_apply(None, None, None, 1, 0, None) == -1
    assert lib.mfs_apply_static(None, None, None, 1, 0, None) == -1
    assert lib.mfs_ghat_apply(None, None, None, 1, 0, None) == -1
    assert lib.mfs_eval_field(None, None, 1, None, 0, None, 0, None) == -1
    assert lib.mfs_solve(None, None, 1, None, None, None, None) == -1
    assert lib.mfs_scene_destroy(None) == 0
    # null descriptor for build_S
    kk = ctypes.c_int64(0)
    assert lib.mfs_build_S(None, None, None, ctypes.byref(kk), None, None, None) == -1
    # descriptor with n > m
    pts = np.zeros((4, 2))
    d = mfs.ShapeDesc(dim=2, kappa=1.0, colloc=pts.ctypes.data, m=2, src=pts.ctypes.data, n=3,
                      proxy=pts.ctypes.data, p=4, eqpts=pts.ctypes.data, k=2, eps_skel=1e-10, eps_ls=1e-13, k_cap=0)
    assert lib.mfs_build_S(ctypes.byref(d), ctypes.c_void_p(1), None, ctypes.byref(kk), None, None, None) == -1


def test_timing_interface_without_device(lib):
    assert lib.mfs_timing_enable(1) == 0
    ms, n, pairs = mfs.timing_read(mfs.MFS_KERNEL_PAIR_F32)
    assert (ms, n, pairs) == (0.0, 0, 0.0)
    assert lib.mfs_timing_enable(0) == 0


def test_pool_interface_without_device(lib):
    st = mfs.pool_stats()
    assert set(st) == {"hits", "misses", "cached_bytes", "live_bytes", "limit_bytes"}
    assert st["limit_bytes"] > 0 and st["cached_bytes"] >= 0
    assert lib.mfs_pool_set_limit(-1) == -1
    mfs.pool_set_limit(st["limit_bytes"])
    mfs.pool_trim()
    assert lib.mfs_pool_query(None) == -1


def test_symmetric_slice_budget_without_device(lib):
    default = 4 << 30
    assert mfs.sym_slice_budget(12345) == default  # the default was in force
    assert mfs.sym_slice_budget(0) == 12345
    assert mfs.sym_slice_budget(-7) == default      # 0 restored the default; so does a negative value
    assert lib.mfs_sym_slice_budget(0, None) == 0   # the previous value is optional


def test_reconstruction_entry_points_reject_null_arguments(lib):
    h = ctypes.c_void_p(0)
    assert lib.mfs_recon_create(None, 1.0, ctypes.byref(h), None) == -1
    pts = np.zeros((4, 2))
    d = mfs.ShapeDesc(dim=2, kappa=1.0, colloc=pts.ctypes.data, m=4, src=pts.ctypes.data, n=2,
                      proxy=pts.ctypes.data, p=4, eqpts=pts.ctypes.data, k=2, eps_skel=1e-10, eps_ls=1e-13, k_cap=0)
    assert lib.mfs_recon_create(ctypes.byref(d), 0.0, ctypes.byref(h), None) == -1   # psi_radius
    assert b"psi_radius" in lib.mfs_last_error()
    assert lib.mfs_recon_destroy(None) == 0
    assert lib.mfs_recon_size(None, None, None, None, None) == -1
    assert lib.mfs_near_sizes(None, None, None, None) == -1
    assert lib.mfs_reconstruct(None, None, None, None, 1, None, None) == -1
    assert lib.mfs_eval_field_near(None, None, None, None, 1, None, 0, None, None) == -1
    assert lib.mfs_plane_wave_colloc(None, None, None, 1, None, None) == -1


def test_scene_rejects_improper_rotation_without_device(lib):
    out = ctypes.c_void_p(0)
    k = np.array([4], np.int64)
    shape_of = np.zeros(1, np.int32)
    centres = np.zeros((1, 2))
    reflection = np.array([[[1.0, 0.0], [0.0, -1.0]]])
    tmpl = np.zeros((4, 2))
    tp = (ctypes.c_void_p * 1)(tmpl.ctypes.data)
    sp = (ctypes.c_void_p * 1)(1)  # never dereferenced: validation fails first
    assert lib.mfs_scene_create(2, 1.0, 1, shape_of.ctypes.data, centres.ctypes.data, reflection.ctypes.data, 1,
                                k.ctypes.data, tp, sp, None, ctypes.byref(out)) == -1
    assert b"rotation" in lib.mfs_last_error()


def test_launch_shape_table_round_trip_without_device(lib, tmp_path):
    """The autotuner's process-wide table as a file: save, clear, load; malformed files are rejected
    whole and leave the table as it was."""
    mfs.tune_clear()
    assert mfs.tune_table_size() == 0
    good = tmp_path / "shapes.txt"
    good.write_text("mfs-tune 2\n2 1 1 18 12 1 0\n2 2 64 18 8 0 -1\n3 0 1 16 32 0 1\n")
    mfs.tune_load(str(good))
    assert mfs.tune_table_size() == 3
    saved = tmp_path / "saved.txt"
    mfs.tune_save(str(saved))
    lines = saved.read_text().splitlines()
    assert lines[0] == "mfs-tune 2"
    assert sorted(lines[1:]) == sorted(good.read_text().splitlines()[1:])
    # bad entries: nchunks out of range, bad rhs per thread, bad dim, bad variant, truncated line, no header
    for body in ("mfs-tune 2\n2 1 1 18 2000 1 0\n", "mfs-tune 2\n2 1 1 18 12 3 0\n", "mfs-tune 2\n4 1 1 18 12 1 0\n",
                 "mfs-tune 2\n2 7 1 18 12 1 0\n", "mfs-tune 2\n2 1 1 18 12 1\n", "2 1 1 18 12 1 0\n",
                 "mfs-tune 2\n2 1 4 10 8 2 0\n2 1 0 10 8 2 0\n", "mfs-tune 2\n2 1 1 18 12 1 2\n",
                 "mfs-tune 1\n2 1 1 18 12 1 0\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(body)
        with pytest.raises(mfs.MfsError):
            mfs.tune_load(str(bad))
        assert mfs.tune_table_size() == 3
    with pytest.raises(mfs.MfsError):
        mfs.tune_load(str(tmp_path / "missing.txt"))
    mfs.tune_clear()
    mfs.tune_load(str(saved))
    assert mfs.tune_table_size() == 3
    mfs.tune_clear()
    assert mfs.tune_table_size() == 0
    assert lib.mfs_autotune(None, 1, 2, 1, None, None) == -1
    assert lib.mfs_tune_set(None, 1, 2, 4, 0, -1) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets the C compiler gives
    the struct of the same fields in include/mfs.h (a field added on one side only fails here)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("mfs_shape_desc", mfs.ShapeDesc), ("mfs_solve_opts", mfs.SolveOpts),
             ("mfs_solve_info", mfs.SolveInfo), ("mfs_pool_stats", mfs.PoolStats),
             ("mfs_tune_result", mfs.TuneResult)]
    lines = ['#include "mfs.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
