"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it; the GPU library never does.
It shares no code with the GPU path; both consume the arrays of ``scenegen``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "_oracle.so"

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> Path:
    """Compile oracle.c with gcc (plain C99, OpenMP, IEEE semantics)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build(force=False)
        L = C.CDLL(str(_LIB))
        L.or_scene_new.restype = C.c_void_p
        L.or_scene_new.argtypes = [_ip, _ip, _ip, _fp, C.c_int, C.c_int]
        L.or_scene_free.argtypes = [C.c_void_p]
        for name in ("or_scene_lipschitz", "or_scene_extent"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_void_p]
        L.or_scene_depth.restype = C.c_int
        L.or_scene_depth.argtypes = [C.c_void_p]
        for name in ("or_scene_roi", "or_scene_dop"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_void_p, C.c_int]
        L.or_scene_voi_box.argtypes = [C.c_void_p, _dp, _dp]
        L.or_eval.argtypes = [C.c_void_p, _dp, C.c_int, _dp, C.c_void_p]
        L.or_op.restype = C.c_double
        L.or_op.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.or_pixel_ray.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, _dp]
        L.or_trace.argtypes = [C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp, C.c_int, C.c_double,
                               C.c_double, _dp, _dp, _ip, _lp]
        L.or_march.argtypes = [C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp, C.c_int, C.c_double, _dp]
        L.or_voi_intervals.argtypes = [C.c_void_p, _dp, C.c_int, C.c_int, _dp, _dp, C.c_int, _ip,
                                       C.c_int, _dp]
        L.or_crease_at.restype = C.c_int
        L.or_crease_at.argtypes = [C.c_void_p, _dp]
        L.or_in_voi.restype = C.c_int
        L.or_in_voi.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_prim.restype = C.c_double
        L.or_prim.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_round_half.restype = C.c_double
        L.or_round_half.argtypes = [C.c_double]
        L.or_mlp.restype = C.c_double
        L.or_mlp.argtypes = [_dp, _dp, _dp, C.c_int, C.c_double, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def camera_array(cam) -> np.ndarray:
    return np.array([*cam.eye, *cam.target, *cam.up, cam.vfov_deg], dtype=np.float64)


class OracleScene:
    """Full-tree FP64 field of a scenegen.Scene (or raw arrays)."""

    def __init__(self, scene=None, *, kind=None, left=None, right=None, params=None, root=None):
        if scene is not None:
            kind, left, right, params, root = scene.kind, scene.left, scene.right, scene.params, scene.root
        self.kind = np.ascontiguousarray(kind, dtype=np.int32)
        self.left = np.ascontiguousarray(left, dtype=np.int32)
        self.right = np.ascontiguousarray(right, dtype=np.int32)
        self.params = np.ascontiguousarray(params, dtype=np.float32).reshape(-1, 16)
        self.root = int(root)
        self.n = self.kind.shape[0]
        self._h = lib().or_scene_new(self.kind, self.left, self.right, self.params.ravel(), self.n, self.root)
        if not self._h:
            raise ValueError("oracle rejected the tree")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_scene_free(h)
            self._h = None

    # scene facts
    @property
    def lipschitz(self) -> float:
        return lib().or_scene_lipschitz(self._h)

    @property
    def depth(self) -> int:
        return lib().or_scene_depth(self._h)

    @property
    def extent(self) -> float:
        return lib().or_scene_extent(self._h)

    def roi(self, i: int) -> float:
        return lib().or_scene_roi(self._h, int(i))

    def d_o(self, i: int) -> float:
        return lib().or_scene_dop(self._h, int(i))

    def voi_box(self):
        lo, hi = np.zeros(3), np.zeros(3)
        lib().or_scene_voi_box(self._h, lo, hi)
        return lo, hi

    def prim_ids(self) -> np.ndarray:
        return np.nonzero(self.kind < 16)[0].astype(np.int32)

    # field
    def eval(self, pts, grad: bool = False):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        n = pts.shape[0]
        f = np.empty(n)
        g = np.empty((n, 3)) if grad else None
        lib().or_eval(self._h, pts.ravel(), n, f, g.ctypes.data_as(C.c_void_p) if grad else None)
        return (f, g) if grad else f

    def op(self, i: int, a: float, b: float) -> float:
        return lib().or_op(self._h, int(i), float(a), float(b))

    def prim(self, i: int, x) -> float:
        return lib().or_prim(self._h, int(i), np.ascontiguousarray(x, dtype=np.float64))

    def crease_at(self, x) -> bool:
        """Sharp-crease flag of the point x (two operands of a sharp branch within 1e-6)."""
        return bool(lib().or_crease_at(self._h, np.ascontiguousarray(x, dtype=np.float64)))

    def in_voi(self, i: int, x) -> bool:
        return bool(lib().or_in_voi(self._h, int(i), np.ascontiguousarray(x, dtype=np.float64)))

    # rays
    def trace(self, camera, px, py, off_r: float = 0.0, off_u: float = 0.0):
        """First roots along the rays through pixel-centre coordinates (px, py)."""
        px = np.ascontiguousarray(px, dtype=np.float64)
        py = np.ascontiguousarray(py, dtype=np.float64)
        n = px.shape[0]
        t, nrm = np.empty(n), np.empty((n, 3))
        flag, ev = np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int64)
        lib().or_trace(self._h, camera_array(camera), camera.width, camera.height, px, py, n,
                       float(off_r), float(off_u), t, nrm.ravel(), flag, ev)
        return t, nrm, flag, ev

    def march(self, camera, px, py, dt: float):
        px = np.ascontiguousarray(px, dtype=np.float64)
        py = np.ascontiguousarray(py, dtype=np.float64)
        t = np.empty(px.shape[0])
        lib().or_march(self._h, camera_array(camera), camera.width, camera.height, px, py,
                       px.shape[0], float(dt), t)
        return t

    def voi_intervals(self, camera, px, py, prim_ids=None):
        """Per ray and primitive, the view-depth interval inside its volume of interest."""
        px = np.ascontiguousarray(px, dtype=np.float64)
        py = np.ascontiguousarray(py, dtype=np.float64)
        ids = self.prim_ids() if prim_ids is None else np.ascontiguousarray(prim_ids, dtype=np.int32)
        out = np.empty((px.shape[0], ids.shape[0], 2))
        lib().or_voi_intervals(self._h, camera_array(camera), camera.width, camera.height, px, py,
                               px.shape[0], ids, ids.shape[0], out.ravel())
        return out


def pixel_ray(camera, px: float, py: float) -> np.ndarray:
    d = np.empty(3)
    lib().or_pixel_ray(camera_array(camera), camera.width, camera.height, float(px), float(py), d)
    return d


def round_half(x):
    f = lib().or_round_half
    return np.vectorize(f, otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def mlp(weights, X, T, omega_max: float = 4.0, grad: bool = True, exact: bool = False, over_weight: float = 4.0):
    """FP64 step-predictor MLP: returns (loss, omega[B], grad[1377] or None).
    exact=True skips the internal binary16 roundings."""
    W = np.ascontiguousarray(weights, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 8)
    T = np.ascontiguousarray(T, dtype=np.float64)
    B = X.shape[0]
    om = np.empty(B)
    g = np.empty(1377) if grad else None
    loss = lib().or_mlp(W, X.ravel(), T, B, float(omega_max), int(bool(exact)), float(over_weight),
                        om.ctypes.data_as(C.c_void_p),
                        g.ctypes.data_as(C.c_void_p) if grad else None)
    return loss, om, g


def silhouette_flags(osc: OracleScene, camera, px, py, t_ref, hit_ref, depth_tol: float,
                     offset: float = 1e-4) -> np.ndarray:
    """Near-silhouette rays: one of four parallel rays displaced by +-offset
    along the camera right/up axes changes hit/miss or moves t* by more than
    ten times the depth tolerance."""
    near = np.zeros(px.shape[0], dtype=bool)
    for dr, du in ((offset, 0.0), (-offset, 0.0), (0.0, offset), (0.0, -offset)):
        t, _, flag, _ = osc.trace(camera, px, py, dr, du)
        hit = (flag & 1) != 0
        near |= hit != hit_ref
        both = hit & hit_ref
        near[both] |= np.abs(t[both] - t_ref[both]) > 10 * depth_tol
        near |= (flag & 2) != 0
    return near


def num_threads() -> int:
    return lib().or_num_threads()
