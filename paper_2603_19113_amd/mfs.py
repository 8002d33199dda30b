"""Python binding of libmfs (argument marshalling only).

Every function here converts arguments and calls the C entry point of the same name in
``libmfs.so`` (declared in include/mfs.h).  Device memory comes from PyTorch tensors on a HIP
device and is passed by pointer together with the current stream; no arithmetic of the method
happens in Python.  If the library is not built, ``load`` raises: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmfs.so")

MFS_OK = 0
MFS_FP64, MFS_FP32, MFS_MIXED = 0, 1, 2
_STATUS = {0: "MFS_OK", -1: "MFS_ERR_ARG", -2: "MFS_ERR_NOMEM", -3: "MFS_ERR_HIP", -4: "MFS_ERR_GEOM",
           -5: "MFS_ERR_RANK", -6: "MFS_ERR_NOCONV"}

_lib = None


class MfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class ShapeDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("colloc", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("proxy", ctypes.c_void_p), ("p", ctypes.c_int64),
                ("eqpts", ctypes.c_void_p), ("k", ctypes.c_int64),
                ("eps_skel", ctypes.c_double), ("eps_ls", ctypes.c_double), ("k_cap", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("prec", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("fp64_until", ctypes.c_double), ("use_x0", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("basis32", ctypes.c_int32), ("deflate", ctypes.c_int32),
                ("block", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("n_matvec32", ctypes.c_int32), ("n_matvec64", ctypes.c_int32), ("n_refine", ctypes.c_int32),
                ("n_restart", ctypes.c_int32), ("relres_max", ctypes.c_double), ("t_total_s", ctypes.c_double),
                ("n_reorth", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class PoolStats(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_int64), ("misses", ctypes.c_int64), ("cached_bytes", ctypes.c_int64),
                ("live_bytes", ctypes.c_int64), ("limit_bytes", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("nchunks", ctypes.c_int32), ("rhs_per_thread", ctypes.c_int32), ("ms", ctypes.c_double),
                ("ms_heuristic", ctypes.c_double), ("n_tried", ctypes.c_int32), ("uses_mfma", ctypes.c_int32),
                ("symmetric", ctypes.c_int32), ("ms_plain", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["mfs_last_error", "mfs_version", "mfs_build_S", "mfs_scene_create", "mfs_scene_destroy",
           "mfs_scene_size", "mfs_scene_points", "mfs_plane_wave", "mfs_ghat_apply", "mfs_s_apply", "mfs_apply",
           "mfs_apply_static", "mfs_solve", "mfs_eval_field", "mfs_timing_enable", "mfs_timing_read", "mfs_pool_query",
           "mfs_pool_set_limit", "mfs_pool_trim", "mfs_sym_slice_budget", "mfs_recon_create", "mfs_recon_destroy", "mfs_recon_size",
           "mfs_near_sizes", "mfs_plane_wave_colloc", "mfs_reconstruct", "mfs_eval_field_near", "mfs_autotune",
           "mfs_tune_get", "mfs_tune_set", "mfs_tune_save", "mfs_tune_load", "mfs_tune_clear", "mfs_tune_table_size",
           "mfs_pair_kernel", "mfs_scene_set_split_fp16", "mfs_solve_footprint"]
MFS_KERNEL_PAIR_F32, MFS_KERNEL_PAIR_F64 = 0, 1
# mfs_pair_kernel_kind
MFS_PAIR_F64, MFS_PAIR_F32, MFS_PAIR_F32_SYM, MFS_PAIR_F32_SYM16, MFS_PAIR_MC_F32, MFS_PAIR_MC_F16X3, \
    MFS_PAIR_MC_F64, MFS_PAIR_F32_SYM_SHARED, MFS_PAIR_F32_SYM16_SHARED = range(9)
PAIR_KERNEL_NAMES = {MFS_PAIR_F64: "f64", MFS_PAIR_F32: "f32", MFS_PAIR_F32_SYM: "f32_sym",
                     MFS_PAIR_F32_SYM16: "f32_sym16", MFS_PAIR_MC_F32: "mc_f32", MFS_PAIR_MC_F16X3: "mc_f16x3",
                     MFS_PAIR_MC_F64: "mc_f64", MFS_PAIR_F32_SYM_SHARED: "f32_sym_shared",
                     MFS_PAIR_F32_SYM16_SHARED: "f32_sym16_shared"}


def load(path: str = LIB_PATH):
    """Load libmfs.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmfs.so is not built ({path}); run python -m paper_2603_19113_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mfs_last_error": ([], ctypes.c_char_p),
        "mfs_version": ([], ctypes.c_int),
        "mfs_build_S": ([ctypes.POINTER(ShapeDesc), vp, vp, ctypes.POINTER(i64), vp, vp, vp], ctypes.c_int),
        "mfs_scene_create": ([i32, f64, i64, vp, vp, vp, i32, vp, vp, vp, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "mfs_scene_destroy": ([vp], ctypes.c_int),
        "mfs_scene_size": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)],
                           ctypes.c_int),
        "mfs_scene_points": ([vp, vp], ctypes.c_int),
        "mfs_plane_wave": ([vp, vp, i32, vp, vp], ctypes.c_int),
        "mfs_ghat_apply": ([vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "mfs_s_apply": ([vp, vp, vp, vp, f64, i32, i32, vp], ctypes.c_int),
        "mfs_apply": ([vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "mfs_apply_static": ([vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "mfs_solve": ([vp, vp, i32, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo), vp], ctypes.c_int),
        "mfs_eval_field": ([vp, vp, i32, vp, i64, vp, i32, vp], ctypes.c_int),
        "mfs_timing_enable": ([i32], ctypes.c_int),
        "mfs_timing_read": ([i32, ctypes.POINTER(f64), ctypes.POINTER(i64), ctypes.POINTER(f64)], ctypes.c_int),
        "mfs_pool_query": ([ctypes.POINTER(PoolStats)], ctypes.c_int),
        "mfs_pool_set_limit": ([i64], ctypes.c_int),
        "mfs_sym_slice_budget": ([i64, ctypes.POINTER(i64)], ctypes.c_int),
        "mfs_pool_trim": ([], ctypes.c_int),
        "mfs_recon_create": ([ctypes.POINTER(ShapeDesc), f64, ctypes.POINTER(vp), vp], ctypes.c_int),
        "mfs_recon_destroy": ([vp], ctypes.c_int),
        "mfs_recon_size": ([vp] + [ctypes.POINTER(i64)] * 4, ctypes.c_int),
        "mfs_near_sizes": ([vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "mfs_plane_wave_colloc": ([vp, vp, vp, i32, vp, vp], ctypes.c_int),
        "mfs_reconstruct": ([vp, vp, vp, vp, i32, vp, vp], ctypes.c_int),
        "mfs_eval_field_near": ([vp, vp, vp, vp, i32, vp, i64, vp, vp], ctypes.c_int),
        "mfs_autotune": ([vp, i32, i32, i32, ctypes.POINTER(TuneResult), vp], ctypes.c_int),
        "mfs_tune_get": ([vp, i32, i32] + [ctypes.POINTER(i32)] * 4, ctypes.c_int),
        "mfs_tune_set": ([vp, i32, i32, i32, i32, i32], ctypes.c_int),
        "mfs_tune_save": ([ctypes.c_char_p], ctypes.c_int),
        "mfs_tune_load": ([ctypes.c_char_p], ctypes.c_int),
        "mfs_tune_clear": ([], ctypes.c_int),
        "mfs_tune_table_size": ([ctypes.POINTER(i64)], ctypes.c_int),
        "mfs_pair_kernel": ([vp, i32, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "mfs_scene_set_split_fp16": ([vp, i32], ctypes.c_int),
        "mfs_solve_footprint": ([i32, i64, vp, i32, vp, i32, i32, ctypes.POINTER(SolveOpts), i64,
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(code: int):
    if code != MFS_OK:
        raise MfsError(code, _lib.mfs_last_error().decode())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _host(a: np.ndarray, dtype=np.float64) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------- build_S ---
@dataclass
class BuiltS:
    S64: object        # torch complex128 [k, k] device tensor holding S column-major (use .T for S)
    S32: object        # torch complex64 copy
    k: int
    skel_idx: np.ndarray | None
    diag: np.ndarray

    def matrix64(self):
        """S as a row-major torch view (S[i, j])."""
        return self.S64.T

    def matrix32(self):
        return self.S32.T


def _shape_desc(shape, kappa, eps_ls, paper_mode, eps_skel, k_cap):
    """ShapeDesc for a workloads.ShapeDiscretisation; returns (desc, capacity k, host arrays to keep)."""
    colloc, src, proxy = _host(shape.colloc), _host(shape.src), _host(shape.proxy)
    desc = ShapeDesc()
    desc.dim, desc.kappa = colloc.shape[1], float(kappa)
    desc.colloc, desc.m = colloc.ctypes.data, colloc.shape[0]
    desc.src, desc.n = src.ctypes.data, src.shape[0]
    desc.proxy, desc.p = proxy.ctypes.data, proxy.shape[0]
    desc.eps_skel, desc.eps_ls = float(eps_skel), float(eps_ls)
    if paper_mode:
        kc = int(k_cap if k_cap is not None else min(colloc.shape[0], proxy.shape[0]))
        desc.eqpts, desc.k, desc.k_cap = None, 0, kc
        return desc, kc, (colloc, src, proxy)
    eq = _host(shape.eqpts)
    desc.eqpts, desc.k, desc.k_cap = eq.ctypes.data, eq.shape[0], 0
    return desc, eq.shape[0], (colloc, src, proxy, eq)


def build_S(shape, kappa: float, eps_ls: float = 1e-13, paper_mode: bool = False, eps_skel: float = 1e-10,
            k_cap: int | None = None, stream=None) -> BuiltS:
    """mfs_build_S for a workloads.ShapeDiscretisation (or any object with colloc/src/proxy/eqpts)."""
    import torch

    lib = load()
    desc, cap, _keep = _shape_desc(shape, kappa, eps_ls, paper_mode, eps_skel, k_cap)
    S64 = torch.empty(cap * cap, dtype=torch.complex128, device="cuda")
    S32 = torch.empty(cap * cap, dtype=torch.complex64, device="cuda")
    k_out = ctypes.c_int64(0)
    skel = np.zeros(max(cap, 1), dtype=np.int64)
    diag = np.zeros(4, dtype=np.float64)
    _check(lib.mfs_build_S(ctypes.byref(desc), _ptr(S64), _ptr(S32), ctypes.byref(k_out),
                           skel.ctypes.data if paper_mode else None, diag.ctypes.data, _stream(stream)))
    k = int(k_out.value)
    S64 = S64[: k * k].view(k, k)
    S32 = S32[: k * k].view(k, k)
    return BuiltS(S64=S64, S32=S32, k=k, skel_idx=skel[:k].copy() if paper_mode else None, diag=diag)


# ------------------------------------------------------------------- scene ---
class Scene:
    """Owns an mfs_scene.  S64/S32 are lists of device tensors (column-major k x k storage)."""

    def __init__(self, dim: int, kappa: float, shape_of, centres, templates, S64, S32=None, rotations=None):
        lib = load()
        self._keep = []
        self.dim = int(dim)
        self.kappa = float(kappa)
        shape_of = _host(shape_of, np.int32)
        centres = _host(centres)
        rot = _host(rotations) if rotations is not None else None
        n_shapes = len(templates)
        tmpl = [_host(t) for t in templates]
        k_of = np.array([t.shape[0] for t in tmpl], dtype=np.int64)
        tmpl_ptrs = (ctypes.c_void_p * n_shapes)(*[t.ctypes.data for t in tmpl])
        s64 = (ctypes.c_void_p * n_shapes)(*[s.data_ptr() for s in S64])
        s32 = (ctypes.c_void_p * n_shapes)(*[s.data_ptr() for s in S32]) if S32 is not None else None
        self._keep += [shape_of, centres, tmpl, k_of, list(S64), list(S32) if S32 is not None else None]
        h = ctypes.c_void_p(0)
        self._keep.append(rot)
        _check(lib.mfs_scene_create(self.dim, self.kappa, shape_of.shape[0], shape_of.ctypes.data,
                                    centres.ctypes.data, rot.ctypes.data if rot is not None else None, n_shapes,
                                    k_of.ctypes.data, tmpl_ptrs, s64, s32, ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64(0)
        t = ctypes.c_int64(0)
        b = ctypes.c_size_t(0)
        _check(lib.mfs_scene_size(h, ctypes.byref(n), ctypes.byref(t), ctypes.byref(b)))
        self.N, self.T = int(n.value), int(t.value)

    def size(self):
        n, t, b = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_size_t(0)
        _check(_lib.mfs_scene_size(self.handle, ctypes.byref(n), ctypes.byref(t), ctypes.byref(b)))
        return int(n.value), int(t.value), int(b.value)

    def points(self) -> np.ndarray:
        out = np.empty((self.N, self.dim), dtype=np.float64)
        _check(_lib.mfs_scene_points(self.handle, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.mfs_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scene_create(dim, kappa, shape_of, centres, templates, S64, S32=None) -> Scene:
    return Scene(dim, kappa, shape_of, centres, templates, S64, S32)


def plane_wave(scene: Scene, dirs, vhat, stream=None):
    d = _host(dirs)
    _check(_lib.mfs_plane_wave(scene.handle, d.ctypes.data, d.shape[0], _ptr(vhat), _stream(stream)))


def ghat_apply(scene: Scene, q, t, prec: int = MFS_FP64, stream=None):
    _check(_lib.mfs_ghat_apply(scene.handle, _ptr(q), _ptr(t), q.shape[0], prec, _stream(stream)))


def s_apply(scene: Scene, q, t, y, beta: float, prec: int = MFS_FP64, stream=None):
    _check(_lib.mfs_s_apply(scene.handle, _ptr(q), _ptr(t), _ptr(y), float(beta), t.shape[0], prec,
                            _stream(stream)))


def apply(scene: Scene, q, y, prec: int = MFS_FP64, stream=None):
    _check(_lib.mfs_apply(scene.handle, _ptr(q), _ptr(y), q.shape[0], prec, _stream(stream)))


def apply_static(scene: Scene, q, y, prec: int = MFS_FP64, stream=None):
    """mfs_apply_static: the operator of mfs_apply with its intermediates in the library's static
    per-device scratch array (no allocation)."""
    _check(_lib.mfs_apply_static(scene.handle, _ptr(q), _ptr(y), q.shape[0], prec, _stream(stream)))


# largest intermediate mfs_apply_static accepts (bytes per device), as in mfs.h
STATIC_SCRATCH_BYTES = 64 << 20


def solve(scene: Scene, vhat, qhat, tol=1e-8, maxit=2000, restart=300, max_refine=10, inner_tol=1e-4,
          prec: int = MFS_FP64, verbose: int = 0, fp64_until: float = 0.0, use_x0: bool = False, stream=None,
          raise_on_noconv: bool = True, use_graph: bool = False, basis32: bool = False,
          deflate: bool = False, block: bool = False) -> dict:
    o = SolveOpts(tol=tol, maxit=maxit, restart=restart, max_refine=max_refine, inner_tol=inner_tol, prec=prec,
                  verbose=verbose, fp64_until=fp64_until, use_x0=1 if use_x0 else 0, use_graph=1 if use_graph else 0,
                  basis32=1 if basis32 else 0, deflate=1 if deflate else 0, block=1 if block else 0)
    info = SolveInfo()
    code = _lib.mfs_solve(scene.handle, _ptr(vhat), vhat.shape[0], ctypes.byref(o), _ptr(qhat),
                          ctypes.byref(info), _stream(stream))
    if code != MFS_OK and (raise_on_noconv or code != -6):
        _check(code)
    d = info.as_dict()
    d["status"] = _STATUS.get(code, code)
    return d


def solve_footprint(dim: int, shape_of, k_of_shape, R: int, restart: int, prec: int = MFS_MIXED,
                    block: bool = False, basis32: bool = False, n_targets: int = 0, rotations: bool = False,
                    fp64_until: float = 0.0) -> int:
    """mfs_solve_footprint: device bytes a scene of this layout holds after a solve (and an FP64
    field evaluation at n_targets points).  Host only."""
    so = np.ascontiguousarray(shape_of, dtype=np.int32)
    ks = np.ascontiguousarray(k_of_shape, dtype=np.int64)
    o = SolveOpts(restart=int(restart), prec=int(prec), block=1 if block else 0, basis32=1 if basis32 else 0,
                  fp64_until=float(fp64_until))
    out = ctypes.c_size_t(0)
    _check(load().mfs_solve_footprint(int(dim), so.shape[0], so.ctypes.data, ks.shape[0], ks.ctypes.data,
                                      1 if rotations else 0, int(R), ctypes.byref(o), int(n_targets),
                                      ctypes.byref(out)))
    return int(out.value)


def eval_field(scene: Scene, qhat, targets, u, prec: int = MFS_FP64, stream=None):
    _check(_lib.mfs_eval_field(scene.handle, _ptr(qhat), qhat.shape[0], _ptr(targets), targets.shape[0], _ptr(u),
                               prec, _stream(stream)))


def timing_enable(on: bool):
    _check(load().mfs_timing_enable(1 if on else 0))


def timing_read(kind: int) -> tuple[float, int, float]:
    """(total kernel milliseconds, launches, pair evaluations) recorded for one kernel kind."""
    ms, n, pairs = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_double(0)
    _check(load().mfs_timing_read(kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pairs)))
    return float(ms.value), int(n.value), float(pairs.value)


# --------------------------------------------------------- reconstruction ---
class Recon:
    """Owns an mfs_recon: the reconstruction factors of one shape (Sec. 4.6)."""

    def __init__(self, shape, kappa: float, psi_radius: float | None = None, eps_ls: float = 1e-13,
                 paper_mode: bool = False, eps_skel: float = 1e-10, k_cap: int | None = None, stream=None):
        lib = load()
        desc, _, keep = _shape_desc(shape, kappa, eps_ls, paper_mode, eps_skel, k_cap)
        radius = float(shape.proxy_radius if psi_radius is None else psi_radius)
        h = ctypes.c_void_p(0)
        _check(lib.mfs_recon_create(ctypes.byref(desc), radius, ctypes.byref(h), _stream(stream)))
        del keep
        self.handle = h
        m, n, k, r = (ctypes.c_int64(0) for _ in range(4))
        _check(lib.mfs_recon_size(h, ctypes.byref(m), ctypes.byref(n), ctypes.byref(k), ctypes.byref(r)))
        self.m, self.n, self.k, self.rank = int(m.value), int(n.value), int(k.value), int(r.value)

    def close(self):
        if getattr(self, "handle", None):
            _lib.mfs_recon_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _recon_array(recons):
    return (ctypes.c_void_p * len(recons))(*[r.handle.value for r in recons])


def near_sizes(scene: Scene, recons) -> tuple[int, int]:
    """(sum of collocation points, sum of MFS sources) over the scene's bodies."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(_lib.mfs_near_sizes(scene.handle, _recon_array(recons), ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def plane_wave_colloc(scene: Scene, recons, directions, v, stream=None):
    d = _host(np.atleast_2d(directions))
    _check(_lib.mfs_plane_wave_colloc(scene.handle, _recon_array(recons), d.ctypes.data, d.shape[0], _ptr(v),
                                      _stream(stream)))


def reconstruct(scene: Scene, recons, v_colloc, qhat, qmfs, stream=None):
    _check(_lib.mfs_reconstruct(scene.handle, _recon_array(recons), _ptr(v_colloc), _ptr(qhat), qhat.shape[0],
                                _ptr(qmfs), _stream(stream)))


def eval_field_near(scene: Scene, recons, qhat, qmfs, targets, u, stream=None):
    _check(_lib.mfs_eval_field_near(scene.handle, _recon_array(recons), _ptr(qhat), _ptr(qmfs), qhat.shape[0],
                                    _ptr(targets), targets.shape[0], _ptr(u), _stream(stream)))


# ------------------------------------------------------------------- pool ---
def pool_stats() -> dict:
    """Counters of the library's device allocation cache."""
    out = PoolStats()
    _check(load().mfs_pool_query(ctypes.byref(out)))
    return out.as_dict()


def pool_set_limit(max_cached_bytes: int):
    _check(load().mfs_pool_set_limit(int(max_cached_bytes)))


def sym_slice_budget(nbytes: int) -> int:
    """Set the symmetric kernel's slice budget (bytes; <= 0: the default) and return the previous."""
    prev = ctypes.c_int64(0)
    _check(load().mfs_sym_slice_budget(int(nbytes), ctypes.byref(prev)))
    return int(prev.value)


def pool_trim():
    _check(load().mfs_pool_trim())


# -------------------------------------------------------------- autotuner ---
def autotune(scene: Scene, R: int = 1, prec: int = MFS_MIXED, reps: int = 3, stream=None) -> dict:
    """Time launch shapes of the operator on this scene and keep the fastest (synchronous)."""
    out = TuneResult()
    _check(_lib.mfs_autotune(scene.handle, int(R), int(prec), int(reps), ctypes.byref(out), _stream(stream)))
    return out.as_dict()


def tune_get(scene: Scene, R: int = 1, prec: int = MFS_MIXED) -> dict:
    nch, rt, sym, src = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.mfs_tune_get(scene.handle, int(R), int(prec), ctypes.byref(nch), ctypes.byref(rt), ctypes.byref(sym),
                             ctypes.byref(src)))
    return {"nchunks": nch.value, "rhs_per_thread": rt.value, "symmetric": sym.value,
            "source": {0: "heuristic", 1: "table", 2: "scene"}[src.value]}


def pair_kernel(scene: Scene, R: int = 1, prec: int = MFS_MIXED) -> int:
    """mfs_pair_kernel: the MFS_PAIR_* kernel the pair sum runs for (R, prec) on this scene."""
    kind = ctypes.c_int32()
    _check(_lib.mfs_pair_kernel(scene.handle, int(R), int(prec), ctypes.byref(kind)))
    return kind.value


def set_split_fp16(scene: Scene, enable: bool):
    """mfs_scene_set_split_fp16: FP16 split-operand (True) or FP32 (False) matrix-core products."""
    _check(_lib.mfs_scene_set_split_fp16(scene.handle, 1 if enable else 0))


def tune_set(scene: Scene, R: int, prec: int, nchunks: int, rhs_per_thread: int = 0, symmetric: int = -1):
    _check(_lib.mfs_tune_set(scene.handle, int(R), int(prec), int(nchunks), int(rhs_per_thread), int(symmetric)))


def tune_save(path: str):
    _check(load().mfs_tune_save(os.fsencode(path)))


def tune_load(path: str):
    _check(load().mfs_tune_load(os.fsencode(path)))


def tune_clear():
    _check(load().mfs_tune_clear())


def tune_table_size() -> int:
    n = ctypes.c_int64()
    _check(load().mfs_tune_table_size(ctypes.byref(n)))
    return n.value
