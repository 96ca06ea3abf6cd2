"""Thin ctypes binding of libsynctrace.so (include/st.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device memory and streams come from PyTorch.  There is no fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import weakref
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libsynctrace.so"

ST_OK, ST_E_INVALID, ST_E_TREE, ST_E_CAPACITY, ST_E_NOMEM, ST_E_DEVICE, ST_E_STALE = range(7)
ST_STEP_PLAIN, ST_STEP_OVERRELAX, ST_STEP_LEARNED, ST_STEP_SEGMENT = 0, 1, 2, 3
ST_ABLATION_PARENT_PTR, ST_ABLATION_FAST_PTR = 0, 1

# every symbol include/st.h declares
EXPORTS = (
    "st_status_str", "st_last_error", "st_default_tuning", "st_flatten_blobtree", "st_scene_destroy",
    "st_scene_get_info", "st_build_abuffer", "st_trace", "st_trace_ex", "st_autotune", "st_debug_eval_field",
    "st_debug_prune_tree",
    "st_debug_abuffer", "st_mlp_pack", "st_mlp_forward", "st_mlp_grad", "st_mlp_adam", "st_set_step_model",
    "st_trace_dump", "st_debug_mfma_probe", "st_batch_create", "st_batch_render", "st_batch_stats",
    "st_batch_destroy", "st_batch_autotune", "st_trace_batch", "st_update_primitives", "st_debug_kernel_timing",
    "st_trace_noalloc", "st_debug_sparse_traversal", "st_trace_ablation", "st_train_step_model",
)

MLP_PARAMS = 1377
MLP_FEATURES = 8
MLP_TABLE_WORDS = 59 * 64 + 16


class StError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"st error {code}: {msg}")
        self.code = code


class StNode(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("left", C.c_int32), ("right", C.c_int32), ("p", C.c_float * 16)]


class StCamera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class StTuning(C.Structure):
    _fields_ = [("tile", C.c_int32), ("max_active", C.c_int32), ("sub_depth", C.c_float),
                ("max_new", C.c_int32), ("eps", C.c_float), ("max_steps", C.c_int32),
                ("refine_iters", C.c_int32), ("step_mode", C.c_int32), ("omega", C.c_float),
                ("lipschitz", C.c_float), ("keep_all_entries", C.c_int32), ("probe_step", C.c_float),
                ("reserved", C.c_int32 * 4)]


class StStats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("hits", C.c_uint64), ("unconverged", C.c_uint64),
                ("field_evals", C.c_uint64), ("grad_evals", C.c_uint64),
                ("node_evals", C.c_uint64 * 4), ("grad_node_evals", C.c_uint64 * 4),
                ("steps", C.c_uint64), ("subfrustums", C.c_uint64), ("empty_views", C.c_uint64),
                ("view_nodes", C.c_uint64), ("abuffer_entries", C.c_uint64), ("max_list", C.c_uint64),
                ("max_overlap", C.c_uint64), ("max_active", C.c_uint64), ("wide_tiles", C.c_uint64),
                ("learned_accepted", C.c_uint64), ("learned_rejected", C.c_uint64),
                ("abuffer_binned", C.c_uint64), ("abuffer_candidates", C.c_uint64),
                ("candidate_pixels", C.c_uint64 * 3), ("abuffer_tested", C.c_uint64), ("stalled", C.c_uint64),
                ("smooth_evals", C.c_uint64), ("block_cycles_max", C.c_uint64),
                ("block_cycles_sum", C.c_uint64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if not isinstance(v, int) else int(v)
        return d


class StSceneInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_prims", C.c_int32), ("depth", C.c_int32), ("extent", C.c_float),
                ("lipschitz", C.c_float), ("voi_lo", C.c_float * 3), ("voi_hi", C.c_float * 3),
                ("device_bytes", C.c_uint64), ("abuffer_bytes", C.c_uint64)]


_lib = None

# st_allocator backed by PyTorch's caching allocator: the scene's device
# buffers come from the same pool as the caller's tensors (allocated on the
# stream the library call runs on; freed blocks return to the pool).
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class StAllocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


_torch = None          # set by lib(): torch, imported before the library
_live_scenes = weakref.WeakSet()


def _torch_alloc(nbytes, stream, ctx):
    try:
        return _torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None   # the library reports ST_E_NOMEM


def _torch_free(ptr, stream, ctx):
    try:
        if ptr:
            _torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass   # the allocator is gone (process exit)


def _close_live_scenes():
    """At exit, before torch's own exit handlers: scenes still alive return
    their buffers to the caching allocator while it exists."""
    for s in list(_live_scenes):
        try:
            s.close()
        except Exception:
            pass


# module-level: the callbacks must outlive every scene that holds them
_TORCH_ALLOCATOR = StAllocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built; run paper_2304_09673_amd/build.py "
                              "(there is no CPU fallback)")
        # torch first: its HIP runtime is then the one the library binds to
        # (same soname).  Loaded the other way round, the process would hold
        # two HIP runtimes, and torch's streams and buffers would be foreign
        # to the library's.
        import atexit
        import torch
        global _torch
        _torch = torch
        # registered after torch's own handlers, so it runs before them
        atexit.register(_close_live_scenes)
        L = C.CDLL(str(LIB_PATH))
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.st_status_str.restype = C.c_char_p
        L.st_status_str.argtypes = [C.c_int]
        L.st_last_error.restype = C.c_char_p
        L.st_last_error.argtypes = []
        L.st_default_tuning.argtypes = [C.POINTER(StTuning)]
        L.st_flatten_blobtree.argtypes = [C.POINTER(StNode), i32, i32, C.POINTER(StAllocator), vp, C.POINTER(vp)]
        L.st_scene_destroy.restype = None
        L.st_scene_destroy.argtypes = [vp]
        L.st_scene_get_info.argtypes = [vp, C.POINTER(StSceneInfo)]
        L.st_build_abuffer.argtypes = [vp, C.POINTER(StCamera), C.POINTER(StTuning), vp]
        L.st_trace.argtypes = [vp, C.POINTER(StCamera), vp, vp, C.POINTER(StStats), vp]
        L.st_trace_ex.argtypes = [vp, C.POINTER(StCamera), vp, vp, vp, C.POINTER(StStats), vp]
        L.st_trace_noalloc.argtypes = [vp, C.POINTER(StCamera), vp, vp, C.POINTER(StStats), vp]
        L.st_trace_ablation.argtypes = [vp, C.POINTER(StCamera), i32, vp, vp, C.POINTER(StStats), vp]
        L.st_autotune.argtypes = [vp, C.POINTER(StCamera), C.POINTER(StTuning), i32, C.POINTER(StTuning), C.POINTER(C.c_float), vp]
        L.st_debug_eval_field.argtypes = [vp, vp, i32, vp, i32, vp, vp, C.POINTER(i32), vp, i32, C.POINTER(i32), vp]
        L.st_debug_prune_tree.argtypes = [C.POINTER(StNode), i32, i32, vp, i32, vp, i32, C.POINTER(i32), C.POINTER(C.c_float)]
        L.st_debug_sparse_traversal.argtypes = [C.POINTER(StNode), i32, i32, vp, i32, i32, vp, i32, C.POINTER(i32),
                                                C.POINTER(C.c_float), C.POINTER(i32)]
        L.st_debug_abuffer.argtypes = [vp, vp, sz, vp, sz, C.POINTER(i32), C.POINTER(i64), vp]
        L.st_mlp_pack.argtypes = [vp, vp, vp, vp]
        L.st_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.st_mlp_grad.argtypes = [vp, vp, vp, vp, i32, C.c_float, vp, vp, vp]
        L.st_mlp_adam.argtypes = [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.st_train_step_model.argtypes = [vp, vp, i64, i32, i32, C.c_float, C.c_float, C.c_uint64, vp, vp, vp, vp]
        L.st_set_step_model.argtypes = [vp, vp, vp, vp]
        L.st_trace_dump.argtypes = [vp, C.POINTER(StCamera), vp, vp, vp, vp, i64, C.POINTER(i64), vp]
        L.st_debug_mfma_probe.argtypes = [vp, vp, vp, vp]
        L.st_batch_create.argtypes = [C.POINTER(vp), C.POINTER(StCamera), i32, C.POINTER(StTuning), C.POINTER(vp),
                                      C.POINTER(vp), vp, C.POINTER(vp)]
        L.st_batch_render.argtypes = [vp, i32, vp]
        L.st_batch_stats.argtypes = [vp, C.POINTER(StStats), i32, vp]
        L.st_batch_destroy.restype = None
        L.st_batch_destroy.argtypes = [vp]
        L.st_batch_autotune.argtypes = [C.POINTER(vp), C.POINTER(StCamera), i32, C.POINTER(StTuning), C.POINTER(vp),
                                        C.POINTER(vp), i32, C.POINTER(StTuning), C.POINTER(C.c_float), vp]
        L.st_update_primitives.argtypes = [vp, vp, C.POINTER(StNode), i32, vp]
        L.st_debug_kernel_timing.argtypes = [vp, i32, C.POINTER(C.c_float), C.POINTER(i32)]
        L.st_trace_batch.argtypes = [C.POINTER(vp), C.POINTER(StCamera), i32, C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(StStats), vp]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is C.c_int or name in ("st_default_tuning",):
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(code):
    if code != ST_OK:
        raise StError(code, lib().st_last_error().decode())


def default_tuning(**kw) -> StTuning:
    t = StTuning()
    _check(lib().st_default_tuning(C.byref(t)))
    for k, v in kw.items():
        if not hasattr(t, k):
            raise KeyError(k)
        setattr(t, k, v)
    return t


def make_camera(cam) -> StCamera:
    c = StCamera()
    c.eye[:] = list(map(float, cam.eye))
    c.target[:] = list(map(float, cam.target))
    c.up[:] = list(map(float, cam.up))
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def nodes_from_arrays(kind, left, right, params):
    n = len(kind)
    arr = (StNode * n)()
    params = np.asarray(params, dtype=np.float32).reshape(n, 16)
    for i in range(n):
        arr[i].kind = int(kind[i])
        arr[i].left = int(left[i])
        arr[i].right = int(right[i])
        arr[i].p[:] = params[i].tolist()
    return arr


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Scene:
    """A flattened blobtree on the GPU (st_flatten_blobtree)."""

    def __init__(self, scene=None, *, kind=None, left=None, right=None, params=None, root=None, stream=None,
                 torch_allocator: bool = True):
        """torch_allocator: the scene's device buffers come from PyTorch's caching
        allocator (False: hipMalloc / hipFree inside the library)."""
        if scene is not None:
            kind, left, right, params, root = scene.kind, scene.left, scene.right, scene.params, scene.root
        self._nodes = nodes_from_arrays(kind, left, right, params)
        self.n = len(self._nodes)
        h = C.c_void_p()
        L = lib()
        alloc = C.byref(_TORCH_ALLOCATOR) if torch_allocator else None
        _check(L.st_flatten_blobtree(self._nodes, self.n, int(root), alloc, _stream_ptr(stream), C.byref(h)))
        _live_scenes.add(self)
        self._h = h
        self._cam = None

    def close(self):
        if getattr(self, "_h", None):
            lib().st_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = StSceneInfo()
        _check(lib().st_scene_get_info(self._h, C.byref(i)))
        return {"n_nodes": i.n_nodes, "n_prims": i.n_prims, "depth": i.depth, "extent": i.extent,
                "lipschitz": i.lipschitz, "voi_lo": list(i.voi_lo), "voi_hi": list(i.voi_hi),
                "device_bytes": i.device_bytes, "abuffer_bytes": i.abuffer_bytes}

    def build_abuffer(self, camera, tuning: StTuning | None = None, stream=None):
        self._cam = make_camera(camera)
        _check(lib().st_build_abuffer(self._h, C.byref(self._cam), C.byref(tuning) if tuning else None,
                                      _stream_ptr(stream)))

    def autotune(self, camera, base: StTuning | None = None, reps: int = 3, stream=None):
        """st_autotune: returns (chosen tuning, its build+trace milliseconds); the
        A-buffer is left built with it."""
        self._cam = make_camera(camera)
        out = StTuning()
        ms = C.c_float(0)
        _check(lib().st_autotune(self._h, C.byref(self._cam), C.byref(base) if base else None, int(reps),
                                 C.byref(out), C.byref(ms), _stream_ptr(stream)))
        return out, float(ms.value)

    def trace(self, camera=None, depth=None, normal=None, stats: bool = True, stream=None, info=None):
        """Returns (depth[H,W], normal[H,W,3], stats dict or None) as torch CUDA tensors.
        info: optional int32/uint32 CUDA tensor [H,W] receiving the per-pixel record."""
        import torch
        cam = make_camera(camera) if camera is not None else self._cam
        W, H = cam.width, cam.height
        if depth is None:
            depth = torch.empty((H, W), dtype=torch.float32, device="cuda")
        if normal is None:
            normal = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        assert depth.is_cuda and depth.dtype == torch.float32 and depth.numel() == H * W and depth.is_contiguous()
        assert normal.is_cuda and normal.dtype == torch.float32 and normal.numel() == 3 * H * W and normal.is_contiguous()
        if info is not None:
            assert info.is_cuda and info.element_size() == 4 and info.numel() == H * W and info.is_contiguous()
        st = StStats() if stats else None
        _check(lib().st_trace_ex(self._h, C.byref(cam), C.c_void_p(depth.data_ptr()), C.c_void_p(normal.data_ptr()),
                                 C.c_void_p(info.data_ptr()) if info is not None else None,
                                 C.byref(st) if st is not None else None, _stream_ptr(stream)))
        return depth, normal, (st.as_dict() if st is not None else None)

    def trace_noalloc(self, depth, normal, camera=None, stats: bool = True, stream=None):
        """st_trace_noalloc into caller-allocated float32 CUDA tensors depth [H,W] and
        normal [H,W,3]; returns the stats dict or None.  The library allocates nothing."""
        cam = make_camera(camera) if camera is not None else self._cam
        _f32_cuda(depth, cam.width * cam.height)
        _f32_cuda(normal, 3 * cam.width * cam.height)
        st = StStats() if stats else None
        _check(lib().st_trace_noalloc(self._h, C.byref(cam), _ptr(depth), _ptr(normal),
                                      C.byref(st) if st is not None else None, _stream_ptr(stream)))
        return st.as_dict() if st is not None else None

    def trace_ablation(self, variant, camera=None, depth=None, normal=None, stats: bool = True, stream=None):
        """st_trace_ablation (per-pixel dexel buffer, unsynchronized rays, Algorithm 1 field
        evaluation with parent or fast ancestor pointers).  Returns (depth, normal, stats or None)."""
        import torch
        cam = make_camera(camera) if camera is not None else self._cam
        W, H = cam.width, cam.height
        if depth is None:
            depth = torch.empty((H, W), dtype=torch.float32, device="cuda")
        if normal is None:
            normal = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        _f32_cuda(depth, H * W)
        _f32_cuda(normal, 3 * H * W)
        st = StStats() if stats else None
        _check(lib().st_trace_ablation(self._h, C.byref(cam), int(variant), _ptr(depth), _ptr(normal),
                                       C.byref(st) if st is not None else None, _stream_ptr(stream)))
        return depth, normal, (st.as_dict() if st is not None else None)

    def debug_eval(self, pts, active=None, grad: bool = False, stream=None):
        """Pruned field f_A of the active primitives (caller node indices, None = all) at
        points (n,3).  Returns (f, grad or None, root_used, device view as caller indices)."""
        import torch
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float32)).cuda()
        n = p.shape[0]
        f = torch.empty(n, dtype=torch.float32, device="cuda")
        g = torch.empty((n, 3), dtype=torch.float32, device="cuda") if grad else None
        used = C.c_int32(0)
        vlen = C.c_int32(0)
        view = np.zeros(2048, dtype=np.int32)
        if active is None:
            a_ptr, na = None, 0
        else:
            a = np.ascontiguousarray(active, dtype=np.int32)
            a_ptr, na = a.ctypes.data_as(C.c_void_p), a.shape[0]
        _check(lib().st_debug_eval_field(self._h, a_ptr, na, C.c_void_p(p.data_ptr()), n, C.c_void_p(f.data_ptr()),
                                         C.c_void_p(g.data_ptr()) if grad else None, C.byref(used),
                                         view.ctypes.data_as(C.c_void_p), view.shape[0], C.byref(vlen),
                                         _stream_ptr(stream)))
        return f, g, int(used.value), view[: vlen.value].copy()

    def update_primitives(self, ids, kind, params, stream=None):
        """st_update_primitives: ids (caller node indices), kind[n], params [n, 16]."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        n = ids.shape[0]
        nodes = nodes_from_arrays(kind, [-1] * n, [-1] * n, params)
        _check(lib().st_update_primitives(self._h, ids.ctypes.data_as(C.c_void_p), nodes, n, _stream_ptr(stream)))

    def set_step_model(self, weights, norm, stream=None):
        """st_set_step_model: weights float32 CUDA [1377], norm float32 CUDA [16]."""
        _f32_cuda(weights, MLP_PARAMS)
        _f32_cuda(norm, 16)
        _check(lib().st_set_step_model(self._h, _ptr(weights), _ptr(norm), _stream_ptr(stream)))

    def trace_dump(self, features, targets, camera=None, depth=None, normal=None, stream=None):
        """st_trace_dump into float32 CUDA tensors features [cap, 8] and targets [cap].
        Returns (samples produced, depth, normal)."""
        import torch
        cam = make_camera(camera) if camera is not None else self._cam
        W, H = cam.width, cam.height
        if depth is None:
            depth = torch.empty((H, W), dtype=torch.float32, device="cuda")
        if normal is None:
            normal = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        _f32_cuda(depth, H * W)
        _f32_cuda(normal, 3 * H * W)
        cap = targets.numel()
        _f32_cuda(targets, cap)
        _f32_cuda(features, 8 * cap)
        n = C.c_int64(0)
        _check(lib().st_trace_dump(self._h, C.byref(cam), _ptr(depth), _ptr(normal), _ptr(features), _ptr(targets),
                                   cap, C.byref(n), _stream_ptr(stream)))
        return int(n.value), depth, normal

    def kernel_timing(self, enable: bool):
        """st_debug_kernel_timing: start recording tile-test launches (enable) or
        stop and return (total milliseconds, launches)."""
        ms, n = C.c_float(0), C.c_int32(0)
        _check(lib().st_debug_kernel_timing(self._h, 1 if enable else 0, C.byref(ms), C.byref(n)))
        return None if enable else (float(ms.value), int(n.value))

    def debug_abuffer(self, stream=None):
        """(tile_off[T+1], node[E], z_in[E], z_out[E]) of the current A-buffer (host numpy)."""
        nt, ne = C.c_int32(0), C.c_int64(0)
        _check(lib().st_debug_abuffer(self._h, None, 0, None, 0, C.byref(nt), C.byref(ne), _stream_ptr(stream)))
        off = np.zeros(nt.value + 1, dtype=np.uint32)
        ent = np.zeros(3 * max(ne.value, 1), dtype=np.uint32)
        _check(lib().st_debug_abuffer(self._h, off.ctypes.data_as(C.c_void_p), off.shape[0],
                                      ent.ctypes.data_as(C.c_void_p), ent.shape[0], C.byref(nt), C.byref(ne),
                                      _stream_ptr(stream)))
        e = ent[: 3 * ne.value].reshape(-1, 3)
        return off, e[:, 0].astype(np.int64), e[:, 1].view(np.float32), e[:, 2].view(np.float32)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _f32_cuda(t, numel):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == numel):
        raise ValueError(f"expected a contiguous float32 CUDA tensor of {numel} elements")


def mlp_pack(weights, norm, table=None, stream=None):
    """st_mlp_pack -> packed table (int32 CUDA tensor [MLP_TABLE_WORDS])."""
    import torch
    _f32_cuda(weights, MLP_PARAMS)
    _f32_cuda(norm, 16)
    if table is None:
        table = torch.empty(MLP_TABLE_WORDS, dtype=torch.int32, device="cuda")
    _check(lib().st_mlp_pack(_ptr(weights), _ptr(norm), _ptr(table), _stream_ptr(stream)))
    return table


def mlp_forward(table, x, out=None, stream=None):
    """st_mlp_forward: omega of raw features x [n, 8] (float32 CUDA)."""
    import torch
    n = x.numel() // 8
    _f32_cuda(x, 8 * n)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device="cuda")
    _f32_cuda(out, n)
    _check(lib().st_mlp_forward(_ptr(table), _ptr(x), n, _ptr(out), _stream_ptr(stream)))
    return out


def mlp_grad(weights, norm, x, target, grad=None, loss=None, over_weight=4.0, stream=None):
    """st_mlp_grad -> (grad [1377], loss [1]) CUDA tensors."""
    import torch
    n = target.numel()
    _f32_cuda(weights, MLP_PARAMS)
    _f32_cuda(norm, 16)
    _f32_cuda(x, 8 * n)
    _f32_cuda(target, n)
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().st_mlp_grad(_ptr(weights), _ptr(norm), _ptr(x), _ptr(target), n, float(over_weight), _ptr(grad), _ptr(loss),
                             _stream_ptr(stream)))
    return grad, loss


def mlp_adam(w, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """st_mlp_adam: in-place update of w, m, v (float32 CUDA, same size)."""
    n = w.numel()
    for t in (w, m, v, grad):
        _f32_cuda(t, n)
    _check(lib().st_mlp_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(grad), n, int(step), float(lr), float(beta1),
                             float(beta2), float(eps), _stream_ptr(stream)))


def train_step_model(x, target, epochs=8, batch=8192, lr=3e-3, over_weight=4.0, seed=0, stream=None):
    """st_train_step_model on float32 CUDA tensors x [n, 8] and target [n];
    returns (weights [1377], norm [16] CUDA tensors, losses per epoch)."""
    import torch
    n = target.numel()
    _f32_cuda(x, 8 * n)
    _f32_cuda(target, n)
    w = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    norm = torch.empty(16, dtype=torch.float32, device="cuda")
    losses = np.zeros(int(epochs), dtype=np.float32)
    _check(lib().st_train_step_model(_ptr(x), _ptr(target), int(n), int(epochs), int(batch), float(lr),
                                     float(over_weight), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(w), _ptr(norm),
                                     losses.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
    return w, norm, losses.astype(np.float64).tolist()


def debug_mfma_probe(a, b, stream=None):
    """st_debug_mfma_probe: D [32, 32] = A [32, 8] . B [8, 32] (float32 CUDA)."""
    import torch
    _f32_cuda(a, 256)
    _f32_cuda(b, 256)
    d = torch.empty((32, 32), dtype=torch.float32, device="cuda")
    _check(lib().st_debug_mfma_probe(_ptr(a), _ptr(b), _ptr(d), _stream_ptr(stream)))
    return d


class Batch:
    """Many scenes rendered per frame by one graph launch (st_batch_*).  Owns
    its output tensors (depths[i] [H,W], normals[i] [H,W,3]); the Scene
    objects must stay alive while the batch exists."""

    def __init__(self, scenes, cameras, tuning: StTuning | None = None, stream=None, autotune: bool = False,
                 reps: int = 2):
        import torch
        self.scenes = list(scenes)
        n = len(self.scenes)
        self._cams = (StCamera * n)(*[make_camera(c) for c in cameras])
        self.depths = [torch.empty((c.height, c.width), dtype=torch.float32, device="cuda") for c in self._cams]
        self.normals = [torch.empty((c.height, c.width, 3), dtype=torch.float32, device="cuda") for c in self._cams]
        self._hs = (C.c_void_p * n)(*[sc._h.value for sc in self.scenes])
        self._dp = (C.c_void_p * n)(*[d.data_ptr() for d in self.depths])
        self._np = (C.c_void_p * n)(*[x.data_ptr() for x in self.normals])
        self.tune_ms = None
        if autotune:
            out = StTuning()
            ms = C.c_float(0)
            _check(lib().st_batch_autotune(self._hs, self._cams, n, C.byref(tuning) if tuning else None, self._dp,
                                           self._np, int(reps), C.byref(out), C.byref(ms), _stream_ptr(stream)))
            tuning, self.tune_ms = out, float(ms.value)
        self.tuning = tuning if tuning is not None else default_tuning()
        h = C.c_void_p()
        _check(lib().st_batch_create(self._hs, self._cams, n, C.byref(self.tuning), self._dp, self._np,
                                     _stream_ptr(stream), C.byref(h)))
        self._h = h

    def render(self, use_graph: bool = True, stream=None):
        _check(lib().st_batch_render(self._h, int(bool(use_graph)), _stream_ptr(stream)))

    def stats(self, stream=None):
        n = len(self.scenes)
        arr = (StStats * n)()
        _check(lib().st_batch_stats(self._h, arr, n, _stream_ptr(stream)))
        return [a.as_dict() for a in arr]

    def close(self):
        if getattr(self, "_h", None):
            lib().st_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prune_tree(kind, left, right, params, root, active):
    """Host-only pruned view (st_debug_prune_tree): (caller indices in evaluation order, Lipschitz)."""
    nodes = nodes_from_arrays(kind, left, right, params)
    n = len(nodes)
    a = np.ascontiguousarray(active if active is not None else [], dtype=np.int32)
    cap = 2 * n + 2
    out = np.zeros(cap, dtype=np.int32)
    ln = C.c_int32(0)
    lip = C.c_float(0)
    _check(lib().st_debug_prune_tree(nodes, n, int(root), a.ctypes.data_as(C.c_void_p) if active is not None else None,
                                     a.shape[0], out.ctypes.data_as(C.c_void_p), cap, C.byref(ln), C.byref(lip)))
    return out[: ln.value].copy(), float(lip.value)


def sparse_traversal(kind, left, right, params, root, active, variant):
    """Host-only Algorithm 1 traversal (st_debug_sparse_traversal): (pruned expression as caller
    indices in evaluation order, Lipschitz, operators visited)."""
    nodes = nodes_from_arrays(kind, left, right, params)
    n = len(nodes)
    a = np.ascontiguousarray(active if active is not None else [], dtype=np.int32)
    cap = 2 * n + 2
    out = np.zeros(cap, dtype=np.int32)
    ln = C.c_int32(0)
    lip = C.c_float(0)
    vis = C.c_int32(0)
    _check(lib().st_debug_sparse_traversal(nodes, n, int(root),
                                           a.ctypes.data_as(C.c_void_p) if active is not None else None,
                                           a.shape[0], int(variant), out.ctypes.data_as(C.c_void_p), cap,
                                           C.byref(ln), C.byref(lip), C.byref(vis)))
    return out[: ln.value].copy(), float(lip.value), int(vis.value)
