"""Python binding of the MI355X Gaussian-splatting rasterizer (``libgsmi.so``).

Argument marshalling only: every step of the render runs in the HIP kernels
behind the C ABI of ``include/gsmi.h``.  PyTorch provides device memory and
the current stream.  The library must be built first
(``python -m paper_2607_15951_amd.build``); importing this module without it
raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgsmi.so")

GS_OK, GS_ERR_INVALID_ARGUMENT, GS_ERR_OUT_OF_MEMORY, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = range(6)
GS_F32, GS_BF16, GS_F16 = 0, 1, 2
PROFILE_STAGES, PROFILE_BLEND_WORK = 1, 2
RENDER_REUSE_ORDER, RENDER_REUSE_LISTS = 1, 2
TILE = 16

EXPORTED = ["gs_create", "gs_destroy", "gs_last_error", "gs_validate", "gs_render", "gs_get_list_info",
            "gs_copy_lists", "gs_copy_projection", "gs_set_profiling", "gs_get_stage_times",
            "gs_get_blend_stats", "gs_get_blend_tile_work", "gs_render_batched", "gs_graph_create",
            "gs_graph_set_views", "gs_graph_launch", "gs_graph_destroy", "gs_render_backward", "gs_set_tuning",
            "gs_get_tuning", "gs_autotune", "gs_get_order_reuse", "gs_render_noalloc",
            "gs_get_list_reuse"]
STAGES = ["project", "depth_sort", "bin_row_count", "bin_row_scatter", "bin_tile_count", "bin_tile_scatter",
          "blend"]


class GsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gsmi status {status}: {message}")
        self.status = status


class gs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("attr_dtype", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class gs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float)]


class gs_render_opts(C.Structure):
    _fields_ = [("background", C.c_float * 3), ("tile_size", C.c_int32), ("pair_capacity", C.c_uint64),
                ("flags", C.c_uint32)]


class gs_list_info(C.Structure):
    _fields_ = [("num_pairs", C.c_uint64), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("n_visible", C.c_int64), ("num_row_entries", C.c_uint64), ("num_tiles", C.c_int64),
                ("num_views", C.c_int32)]


class gs_gradients(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class gs_tuning(C.Structure):
    _fields_ = [("sort_items", C.c_int32), ("bin_row_items", C.c_int32), ("bin_tile_items", C.c_int32),
                ("blend_tile_group", C.c_int32), ("blend_batch", C.c_int32)]


TUNE_CANDIDATES = [("sort_items", v) for v in (4, 8, 16)] + [("bin_row_items", v) for v in (4, 8, 16)] + \
    [("bin_tile_items", v) for v in (8, 16, 32)] + [("blend_tile_group", v) for v in (-1, 0, 1, 2, 4, 8, 16, 32, 64)] + \
    [("blend_batch", v) for v in (128, 256, 512)]


class gs_view(C.Structure):
    _fields_ = [("camera", gs_camera), ("width", C.c_int32), ("height", C.c_int32), ("out_rgb", C.c_void_p),
                ("out_final_T", C.c_void_p), ("out_n_contrib", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libgsmi.so and declares its C signatures (no device call)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2607_15951_amd.build`")
    # PyTorch brings its own HIP runtime under the same soname as the system
    # one the library is linked against: load it first, so that the process
    # has one runtime (the library loaded first would bind PyTorch to the
    # system runtime, where PyTorch then finds no GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    P = C.c_void_p
    L.gs_create.argtypes = [C.c_int, C.POINTER(P)]
    L.gs_create.restype = C.c_int
    L.gs_destroy.argtypes = [P]
    L.gs_destroy.restype = None
    L.gs_last_error.argtypes = [P]
    L.gs_last_error.restype = C.c_char_p
    L.gs_validate.argtypes = [C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.c_int32, C.c_int32,
                              C.POINTER(gs_render_opts), P]
    L.gs_validate.restype = C.c_int
    L.gs_render.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.c_int32, C.c_int32,
                            C.POINTER(gs_render_opts), P, P, P, P]
    L.gs_render.restype = C.c_int
    L.gs_render_noalloc.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(gs_camera), C.c_int32, C.c_int32,
                                    C.POINTER(gs_render_opts), P, P, P, P]
    L.gs_render_noalloc.restype = C.c_int
    L.gs_render_batched.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(gs_view), C.c_int32,
                                    C.POINTER(gs_render_opts), P]
    L.gs_render_batched.restype = C.c_int
    L.gs_graph_create.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(gs_view), C.c_int32,
                                  C.POINTER(gs_render_opts), P, C.POINTER(P)]
    L.gs_graph_create.restype = C.c_int
    L.gs_graph_set_views.argtypes = [P, C.POINTER(gs_view), C.c_int32, P]
    L.gs_graph_set_views.restype = C.c_int
    L.gs_graph_launch.argtypes = [P, P]
    L.gs_graph_launch.restype = C.c_int
    L.gs_graph_destroy.argtypes = [P]
    L.gs_graph_destroy.restype = None
    L.gs_render_backward.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(gs_gradients), P]
    L.gs_render_backward.restype = C.c_int
    L.gs_get_order_reuse.argtypes = [P, C.POINTER(C.c_uint32)]
    L.gs_get_order_reuse.restype = C.c_int
    L.gs_get_list_reuse.argtypes = [P, C.POINTER(C.c_uint32)]
    L.gs_get_list_reuse.restype = C.c_int
    L.gs_set_tuning.argtypes = [P, C.POINTER(gs_tuning)]
    L.gs_set_tuning.restype = C.c_int
    L.gs_get_tuning.argtypes = [P, C.POINTER(gs_tuning)]
    L.gs_get_tuning.restype = C.c_int
    L.gs_autotune.argtypes = [P, C.POINTER(gs_gaussians), C.POINTER(gs_view), C.c_int32, C.POINTER(gs_render_opts),
                              C.c_int32, P, C.POINTER(gs_tuning), C.POINTER(C.c_float)]
    L.gs_autotune.restype = C.c_int
    L.gs_get_list_info.argtypes = [P, C.POINTER(gs_list_info)]
    L.gs_get_list_info.restype = C.c_int
    L.gs_copy_lists.argtypes = [P, P, P, P, P]
    L.gs_copy_lists.restype = C.c_int
    L.gs_copy_projection.argtypes = [P, P, P, P, P, P, P]
    L.gs_copy_projection.restype = C.c_int
    L.gs_set_profiling.argtypes = [P, C.c_int32]
    L.gs_set_profiling.restype = C.c_int
    L.gs_get_stage_times.argtypes = [P, C.POINTER(C.c_float), C.c_int32]
    L.gs_get_stage_times.restype = C.c_int
    L.gs_get_blend_stats.argtypes = [P, C.POINTER(C.c_uint64)]
    L.gs_get_blend_stats.restype = C.c_int
    L.gs_get_blend_tile_work.argtypes = [P, C.POINTER(C.c_uint64), C.c_int64]
    L.gs_get_blend_tile_work.restype = C.c_int
    _lib = L
    return L


def make_camera(cam: dict) -> gs_camera:
    c = gs_camera()
    R = np.asarray(cam["R"], np.float32).reshape(9)
    t = np.asarray(cam["t"], np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    c.near_plane = float(np.float32(cam["near"]))
    return c


def make_opts(background=(0.0, 0.0, 0.0), pair_capacity: int = 0, flags: int = 0) -> gs_render_opts:
    o = gs_render_opts()
    for k in range(3):
        o.background[k] = float(background[k])
    o.tile_size = TILE
    o.pair_capacity = int(pair_capacity)
    o.flags = int(flags)
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _torch():
    import torch
    return torch


def scene_to_device(scene: dict, dtype: int = GS_F32, device="cuda"):
    """Uploads a scenes.make_scene() dict; non-mean attributes in ``dtype``."""
    torch = _torch()
    tdt = {GS_F32: torch.float32, GS_BF16: torch.bfloat16, GS_F16: torch.float16}[dtype]
    out = {"sh_degree": int(scene["sh_degree"]), "attr_dtype": dtype,
           "means": torch.from_numpy(np.ascontiguousarray(scene["means"], np.float32)).to(device)}
    for k in ("log_scales", "quats", "opacity_logits", "sh"):
        t = torch.from_numpy(np.ascontiguousarray(scene[k], np.float32))
        out[k] = t.to(tdt).contiguous().to(device)
    return out


def _check_tensor(t, name: str, shape: tuple, dtype, device):
    """The C ABI takes bare device pointers and cannot see a tensor's device,
    dtype, layout or size: they are checked here, before any call."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a cuda tensor (got {t.device})")
    if t.device != device:
        raise ValueError(f"{name} must live on {device} (got {t.device})")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _attr_torch_dtype(attr_dtype: int):
    torch = _torch()
    return {GS_F32: torch.float32, GS_BF16: torch.bfloat16, GS_F16: torch.float16}[attr_dtype]


def make_gaussians(dev_scene: dict) -> gs_gaussians:
    torch = _torch()
    means = dev_scene["means"]
    if not isinstance(means, torch.Tensor) or means.dim() != 2 or means.shape[0] != 3:
        raise ValueError("means must be a [3, n] tensor")
    n = int(means.shape[1])
    deg = int(dev_scene["sh_degree"])
    attr = int(dev_scene.get("attr_dtype", GS_F32))
    if deg not in (0, 1, 2, 3) or attr not in (GS_F32, GS_BF16, GS_F16):
        raise ValueError("sh_degree must be 0..3 and attr_dtype GS_F32, GS_BF16 or GS_F16")
    adt = _attr_torch_dtype(attr)
    _check_tensor(means, "means", (3, n), torch.float32, means.device)
    for k, shape in (("log_scales", (3, n)), ("quats", (4, n)), ("opacity_logits", (n,)),
                     ("sh", ((deg + 1) ** 2, 3, n))):
        _check_tensor(dev_scene[k], k, shape, adt, means.device)
    g = gs_gaussians()
    g.n = n
    g.sh_degree = deg
    g.attr_dtype = attr
    g.means = dev_scene["means"].data_ptr()
    g.log_scales = dev_scene["log_scales"].data_ptr()
    g.quats = dev_scene["quats"].data_ptr()
    g.opacity_logits = dev_scene["opacity_logits"].data_ptr()
    g.sh = dev_scene["sh"].data_ptr()
    return g


def validate(gaussians: gs_gaussians, camera: gs_camera, width: int, height: int,
             opts: gs_render_opts | None, out_rgb_ptr) -> int:
    """Host-only argument check (no device touched); returns the status code."""
    L = load_library()
    return int(L.gs_validate(C.byref(gaussians), C.byref(camera), int(width), int(height),
                             C.byref(opts) if opts is not None else None, out_rgb_ptr))


def _check_outputs(out: dict, width: int, height: int, device):
    """Caller-given output tensors of one view: rgb [3,H,W] float32, final_T
    [H,W] float32 or None, n_contrib [H,W] int32 or None."""
    torch = _torch()
    _check_tensor(out["image"], "image", (3, height, width), torch.float32, device)
    if out.get("final_T") is not None:
        _check_tensor(out["final_T"], "final_T", (height, width), torch.float32, device)
    if out.get("n_contrib") is not None:
        _check_tensor(out["n_contrib"], "n_contrib", (height, width), torch.int32, device)


class Renderer:
    """One gs_context on one device.  Not thread-safe."""

    def __init__(self, device: int = 0):
        self._L = load_library()
        self._ctx = C.c_void_p()
        st = self._L.gs_create(int(device), C.byref(self._ctx))
        if st != GS_OK:
            raise GsError(st, self._L.gs_last_error(None).decode())
        self.device = device
        self._last = None
        self._graphs = []   # live RenderGraphs: closed before the context
        self.generation = 0   # counts renders: a pending backward needs the latest one

    def close(self):
        for gr in list(self._graphs):
            gr.close()
        if self._ctx:
            self._L.gs_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != GS_OK:
            raise GsError(st, self._L.gs_last_error(self._ctx).decode())

    def render(self, dev_scene: dict, camera: dict, width: int, height: int, background=(0.0, 0.0, 0.0),
               pair_capacity: int = 0, out=None, want_T: bool = True, want_n_contrib: bool = True,
               stream=None, reuse_order: bool = False, reuse_lists: bool = False):
        """Renders into (new or given) tensors: rgb [3,H,W], final_T [H,W], n_contrib [H,W].
        reuse_order: start the depth sort from the previous render's order
        (GS_RENDER_REUSE_ORDER; same results, less work between nearby frames).
        reuse_lists: keep the previous render's tile lists when no Gaussian's
        depth key or tile rectangle changed (GS_RENDER_REUSE_LISTS; same
        results, no sort and no binning for a static camera)."""
        torch = _torch()
        dev = dev_scene["means"].device
        if out is None:
            out = {"image": torch.empty((3, height, width), dtype=torch.float32, device=dev),
                   "final_T": torch.empty((height, width), dtype=torch.float32, device=dev) if want_T else None,
                   "n_contrib": torch.empty((height, width), dtype=torch.int32, device=dev)
                   if want_n_contrib else None}
        else:
            _check_outputs(out, int(width), int(height), dev)
        g = make_gaussians(dev_scene)
        cam = make_camera(camera)
        flags = (RENDER_REUSE_ORDER if reuse_order else 0) | (RENDER_REUSE_LISTS if reuse_lists else 0)
        opts = make_opts(background, pair_capacity, flags)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        st = self._L.gs_render(self._ctx, C.byref(g), C.byref(cam), int(width), int(height), C.byref(opts),
                               _ptr(out["image"]), _ptr(out.get("final_T")), _ptr(out.get("n_contrib")),
                               C.c_void_p(s))
        self._check(st)
        self._last = (dev, int(g.n))
        # the backward reads these outputs: hold them so that the caching
        # allocator does not hand their memory to another tensor meanwhile
        self._last_out = out
        self.generation += 1
        return out

    def render_noalloc(self, dev_scene: dict, camera: dict, width: int, height: int, out: dict,
                       background=(0.0, 0.0, 0.0), pair_capacity: int = 0, stream=None):
        """gs_render_noalloc into the caller's output tensors (which the
        caller allocates beforehand: the library allocates nothing here)."""
        torch = _torch()
        dev = dev_scene["means"].device
        _check_outputs(out, int(width), int(height), dev)
        g = make_gaussians(dev_scene)
        cam = make_camera(camera)
        opts = make_opts(background, pair_capacity)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        self._check(self._L.gs_render_noalloc(self._ctx, C.byref(g), C.byref(cam), int(width), int(height),
                                              C.byref(opts), _ptr(out["image"]), _ptr(out.get("final_T")),
                                              _ptr(out.get("n_contrib")), C.c_void_p(s)))
        self._last = (dev, int(g.n))
        self._last_out = None   # nothing of this render can be differentiated
        self.generation += 1
        return out

    def render_batched(self, dev_scene: dict, cameras: list, background=(0.0, 0.0, 0.0), pair_capacity: int = 0,
                       outs=None, want_T: bool = True, want_n_contrib: bool = True, stream=None,
                       reuse_lists: bool = False):
        """Renders every camera dict of ``cameras`` (each with its own
        width/height) in one gs_render_batched call; returns one output dict
        per view, as render() does.  reuse_lists: GS_RENDER_REUSE_LISTS."""
        torch = _torch()
        dev = dev_scene["means"].device
        views, outs = self._views(cameras, outs, dev, want_T, want_n_contrib)
        g = make_gaussians(dev_scene)
        opts = make_opts(background, pair_capacity, RENDER_REUSE_LISTS if reuse_lists else 0)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        self._check(self._L.gs_render_batched(self._ctx, C.byref(g), views, len(cameras), C.byref(opts),
                                              C.c_void_p(s)))
        self._last = (dev, int(g.n) * len(cameras))
        self._last_out = outs
        self.generation += 1
        return outs

    def _views(self, cameras, outs, dev, want_T=True, want_n_contrib=True):
        torch = _torch()
        if outs is None:
            outs = []
            for c in cameras:
                W, H = int(c["width"]), int(c["height"])
                outs.append({"image": torch.empty((3, H, W), dtype=torch.float32, device=dev),
                             "final_T": torch.empty((H, W), dtype=torch.float32, device=dev) if want_T else None,
                             "n_contrib": torch.empty((H, W), dtype=torch.int32, device=dev)
                             if want_n_contrib else None})
        else:
            if len(outs) != len(cameras):
                raise ValueError("outs must hold one output dict per camera")
            for c, o in zip(cameras, outs):
                _check_outputs(o, int(c["width"]), int(c["height"]), dev)
        views = (gs_view * len(cameras))()
        for k, (c, o) in enumerate(zip(cameras, outs)):
            views[k].camera = make_camera(c)
            views[k].width, views[k].height = int(c["width"]), int(c["height"])
            views[k].out_rgb = _ptr(o["image"])
            views[k].out_final_T = _ptr(o.get("final_T"))
            views[k].out_n_contrib = _ptr(o.get("n_contrib"))
        return views, outs

    def graph(self, dev_scene: dict, cameras: list, pair_capacity: int, background=(0.0, 0.0, 0.0), outs=None,
              stream=None, reuse_order: bool = False, reuse_lists: bool = False) -> "RenderGraph":
        """Captures a batched render of ``cameras`` into a replayable graph
        (gs_graph_create); the renderer belongs to it until it is closed."""
        torch = _torch()
        dev = dev_scene["means"].device
        views, outs = self._views(cameras, outs, dev)
        g = make_gaussians(dev_scene)
        flags = (RENDER_REUSE_ORDER if reuse_order else 0) | (RENDER_REUSE_LISTS if reuse_lists else 0)
        opts = make_opts(background, pair_capacity, flags)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        h = C.c_void_p()
        self._check(self._L.gs_graph_create(self._ctx, C.byref(g), views, len(cameras), C.byref(opts),
                                            C.c_void_p(s), C.byref(h)))
        self._last = (dev, int(g.n) * len(cameras))
        gr = RenderGraph(self, h, outs, dev)
        self._graphs.append(gr)
        return gr

    def order_reuse(self) -> dict:
        """Outcome of the last render's reuse of the previous depth order
        (gs_get_order_reuse): whether the radix sort was skipped, and the
        descents of the previous order under the new depths."""
        w = (C.c_uint32 * 2)()
        self._check(self._L.gs_get_order_reuse(self._ctx, w))
        return {"reused": bool(w[0]), "descents": int(w[1])}

    def list_reuse(self) -> dict:
        """Outcome of the last render's comparison with the previous lists
        (gs_get_list_reuse): whether the lists were kept (sort and binning
        skipped), and the Gaussians whose depth key or tile rectangle changed."""
        w = (C.c_uint32 * 2)()
        self._check(self._L.gs_get_list_reuse(self._ctx, w))
        return {"reused": bool(w[0]), "changed": int(w[1])}

    def tuning(self) -> dict:
        t = gs_tuning()
        self._check(self._L.gs_get_tuning(self._ctx, C.byref(t)))
        return {k: int(getattr(t, k)) for k, _ in gs_tuning._fields_}

    def set_tuning(self, **kw):
        """Changes launch shapes (gs_set_tuning); unnamed fields keep their value."""
        cur = self.tuning()
        cur.update(kw)
        t = gs_tuning(**cur)
        self._check(self._L.gs_set_tuning(self._ctx, C.byref(t)))

    def autotune(self, dev_scene: dict, cameras: list, reps: int = 3, background=(0.0, 0.0, 0.0),
                 pair_capacity: int = 0, stream=None) -> dict:
        """gs_autotune over a batched render of ``cameras``: returns the chosen
        tuning and the scored milliseconds of every candidate."""
        torch = _torch()
        dev = dev_scene["means"].device
        views, outs = self._views(cameras, None, dev)
        g = make_gaussians(dev_scene)
        opts = make_opts(background, pair_capacity)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        t = gs_tuning()
        ms = (C.c_float * len(TUNE_CANDIDATES))()
        self._check(self._L.gs_autotune(self._ctx, C.byref(g), views, len(cameras), C.byref(opts), int(reps),
                                        C.c_void_p(s), C.byref(t), ms))
        self._last = (dev, int(g.n) * len(cameras))
        self._last_out = outs
        self.generation += 1
        return {"tuning": {k: int(getattr(t, k)) for k, _ in gs_tuning._fields_},
                "candidates_ms": [(name, v, round(float(ms[i]), 4)) for i, (name, v) in enumerate(TUNE_CANDIDATES)]}

    def backward(self, dev_scene: dict, grad_images: list, grad_T: list | None = None, stream=None) -> dict:
        """Gradients of the Gaussian parameters (float32 tensors, input
        layouts) for dL/d(image) of every view of the last render (and
        optionally dL/d(final_T)); see gs_render_backward.  The backward
        reads that render's image, final_T and n_contrib, which must not
        have been written since (the renderer holds a reference to them)."""
        torch = _torch()
        dev = dev_scene["means"].device
        n = dev_scene["means"].shape[1]
        ncoef = dev_scene["sh"].shape[0]
        if self._last is None or self._last[0] != dev:
            raise ValueError("the scene must live where the last render ran")
        for k, t in enumerate(grad_images):
            o = self._last_out[k] if isinstance(self._last_out, list) else self._last_out
            _check_tensor(t.contiguous(), f"grad_images[{k}]", tuple(o["image"].shape), torch.float32, dev)
            if grad_T is not None and grad_T[k] is not None:
                _check_tensor(grad_T[k].contiguous(), f"grad_T[{k}]", tuple(o["image"].shape[1:]), torch.float32,
                              dev)
        out = {"means": torch.empty((3, n), dtype=torch.float32, device=dev),
               "log_scales": torch.empty((3, n), dtype=torch.float32, device=dev),
               "quats": torch.empty((4, n), dtype=torch.float32, device=dev),
               "opacity_logits": torch.empty(n, dtype=torch.float32, device=dev),
               "sh": torch.empty((ncoef, 3, n), dtype=torch.float32, device=dev)}
        gi = [t.contiguous() for t in grad_images]
        gt = [t.contiguous() if t is not None else None for t in grad_T] if grad_T is not None else None
        arr_i = (C.c_void_p * len(gi))(*[_ptr(t) for t in gi])
        arr_t = (C.c_void_p * len(gi))(*[_ptr(t) for t in gt]) if gt is not None else None
        gr = gs_gradients(_ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                          _ptr(out["opacity_logits"]), _ptr(out["sh"]))
        g = make_gaussians(dev_scene)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        self._check(self._L.gs_render_backward(self._ctx, C.byref(g), arr_i, arr_t, C.byref(gr), C.c_void_p(s)))
        return out

    def set_profiling(self, stages: bool = True, blend_work: bool = False):
        """Tracing of the following renders: HIP events between the stages
        (stage_times) and/or the counting variant of the blend (blend_stats)."""
        flags = (PROFILE_STAGES if stages else 0) | (PROFILE_BLEND_WORK if blend_work else 0)
        self._check(self._L.gs_set_profiling(self._ctx, flags))

    def stage_times(self) -> dict:
        """Device milliseconds per stage of the last (timed) render."""
        ms = (C.c_float * len(STAGES))()
        self._check(self._L.gs_get_stage_times(self._ctx, ms, len(STAGES)))
        return {k: float(ms[i]) for i, k in enumerate(STAGES)}

    def blend_stats(self) -> dict:
        """Blend work counters of the last traced render."""
        v = (C.c_uint64 * 4)()
        self._check(self._L.gs_get_blend_stats(self._ctx, v))
        return dict(evaluations=int(v[0]), composited=int(v[1]), staged=int(v[2]), lane_evaluations=int(v[3]))

    def blend_tile_work(self):
        """Per-tile trace of the last counted render: numpy uint64 [tiles, 6]
        (start, end on the 100 MHz device clock, entries staged, wave bodies,
        evaluations, composited)."""
        import numpy as np
        info = self.list_info()
        T = info["num_tiles"]
        buf = (C.c_uint64 * (6 * T))()
        self._check(self._L.gs_get_blend_tile_work(self._ctx, buf, T))
        return np.frombuffer(buf, dtype=np.uint64).reshape(T, 6).copy()

    def list_info(self) -> dict:
        info = gs_list_info()
        self._check(self._L.gs_get_list_info(self._ctx, C.byref(info)))
        return dict(num_pairs=int(info.num_pairs), tiles_x=info.tiles_x, tiles_y=info.tiles_y,
                    n_visible=int(info.n_visible), num_row_entries=int(info.num_row_entries),
                    num_tiles=int(info.num_tiles), num_views=int(info.num_views))

    def lists(self, keys: bool = False) -> dict:
        """Sorted per-tile lists of the last render as device tensors."""
        torch = _torch()
        info = self.list_info()
        dev = self._last[0]
        K = info["num_pairs"]
        T = info["num_tiles"]
        values = torch.empty(max(K, 1), dtype=torch.int32, device=dev)
        offsets = torch.empty(T + 1, dtype=torch.int32, device=dev)
        kt = torch.empty(max(K, 1), dtype=torch.int64, device=dev) if keys else None
        s = torch.cuda.current_stream(dev).cuda_stream
        self._check(self._L.gs_copy_lists(self._ctx, _ptr(values), _ptr(offsets), _ptr(kt), C.c_void_p(s)))
        res = dict(values=values[:K], tile_offsets=offsets, **info)
        if keys:
            res["keys"] = kt[:K]
        return res

    def projection(self) -> dict:
        torch = _torch()
        dev, n = self._last
        n1 = max(n, 1)
        out = dict(splats=torch.empty((n1, 12), dtype=torch.float32, device=dev),
                   depth_key=torch.empty(n1, dtype=torch.int32, device=dev),
                   radius=torch.empty(n1, dtype=torch.int32, device=dev),
                   tiles_touched=torch.empty(n1, dtype=torch.int32, device=dev),
                   rect=torch.empty((n1, 4), dtype=torch.int16, device=dev))
        s = torch.cuda.current_stream(dev).cuda_stream
        self._check(self._L.gs_copy_projection(self._ctx, *[_ptr(out[k]) for k in
                                                            ("splats", "depth_key", "radius", "tiles_touched",
                                                             "rect")], C.c_void_p(s)))
        return {k: v[:n] for k, v in out.items()}


class RenderGraph:
    """A captured batched render (gs_graph_*): launch() replays it, set_views()
    changes cameras and outputs of the same sizes between launches."""

    def __init__(self, renderer: Renderer, handle, outs, dev):
        self._r, self._h, self.outs, self._dev = renderer, handle, outs, dev

    def launch(self, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self._dev).cuda_stream
        self._r._check(self._r._L.gs_graph_launch(self._h, C.c_void_p(s)))
        # a backward now differentiates this launch, whose outputs it reads
        self._r._last_out = self.outs
        self._r.generation += 1
        return self.outs

    def set_views(self, cameras: list, outs=None, stream=None):
        torch = _torch()
        views, outs = self._r._views(cameras, outs if outs is not None else self.outs, self._dev)
        s = stream if stream is not None else torch.cuda.current_stream(self._dev).cuda_stream
        self._r._check(self._r._L.gs_graph_set_views(self._h, views, len(cameras), C.c_void_p(s)))
        self.outs = outs

    def close(self):
        if self._h:
            self._r._L.gs_graph_destroy(self._h)
            self._h = None
            if self in self._r._graphs:
                self._r._graphs.remove(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scene_from_rows(means, log_scales, quats, opacity_logits, sh, attr_dtype: int = GS_F32) -> dict:
    """A device scene in the library's channel-major layout from per-Gaussian
    rows (the common [N, C] layout of 3DGS checkpoints): means [N, 3],
    log_scales [N, 3], quats [N, 4] (w, x, y, z), opacity_logits [N] and sh
    [N, (deg+1)^2, 3] CUDA tensors.  Transposes once per scene (one copy);
    attributes other than the means are stored in ``attr_dtype``."""
    torch = _torch()
    tdt = _attr_torch_dtype(attr_dtype)
    n = means.shape[0]
    if sh.dim() != 3 or sh.shape[0] != n or sh.shape[2] != 3:
        raise ValueError("sh must be [N, (deg+1)^2, 3]")
    deg = int(round(math.sqrt(sh.shape[1]))) - 1
    if (deg + 1) ** 2 != sh.shape[1]:
        raise ValueError("sh must hold (deg+1)^2 coefficients per channel")
    return {"sh_degree": deg, "attr_dtype": attr_dtype,
            "means": means.to(torch.float32).t().contiguous(),
            "log_scales": log_scales.to(tdt).t().contiguous(),
            "quats": quats.to(tdt).t().contiguous(),
            "opacity_logits": opacity_logits.reshape(n).to(tdt).contiguous(),
            "sh": sh.to(tdt).permute(1, 2, 0).contiguous()}


_DEFAULT_RENDERERS = {}


def render(dev_scene: dict, camera: dict, size, background=(0.0, 0.0, 0.0), keys: bool = False,
           renderer: "Renderer | None" = None):
    """One frame, gs_render, on a renderer kept per device: returns (image
    [3, H, W], lists), where lists holds the sorted per-tile lists of the
    frame (Sec. 3.1) as device tensors: values [K], tile_offsets [T + 1] (tile
    t's list is values[tile_offsets[t]:tile_offsets[t + 1]]), keys [K] with
    keys=True, and the sizes of gs_get_list_info."""
    torch = _torch()
    width, height = (int(v) for v in size)
    dev = dev_scene["means"].device
    if renderer is None:
        key = dev.index if dev.index is not None else torch.cuda.current_device()
        renderer = _DEFAULT_RENDERERS.get(key)
        if renderer is None:
            renderer = _DEFAULT_RENDERERS[key] = Renderer(key)
    out = renderer.render(dev_scene, camera, width, height, background=background)
    return out["image"], renderer.lists(keys=keys)


def render_autograd(renderer: Renderer, means, log_scales, quats, opacity_logits, sh, camera: dict, width: int,
                    height: int, background=(0.0, 0.0, 0.0)):
    """Differentiable render: (image [3,H,W], final_T [H,W]) with gradients
    to the float32 parameter tensors through gs_render_backward.  The
    renderer must not render again before the backward of this call."""
    return _RenderFunction.apply(renderer, camera, int(width), int(height), tuple(background), means, log_scales,
                                 quats, opacity_logits, sh)


def _autograd_function():
    torch = _torch()

    class RenderFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, renderer, camera, width, height, background, means, log_scales, quats, opacity_logits, sh):
            ncoef = sh.shape[0]
            deg = {1: 0, 4: 1, 9: 2, 16: 3}[ncoef]
            scene = {"means": means.detach().contiguous(), "log_scales": log_scales.detach().contiguous(),
                     "quats": quats.detach().contiguous(), "opacity_logits": opacity_logits.detach().contiguous(),
                     "sh": sh.detach().contiguous(), "sh_degree": deg, "attr_dtype": GS_F32}
            out = renderer.render(scene, camera, width, height, background=background)
            ctx.renderer, ctx.scene, ctx.generation = renderer, scene, renderer.generation
            # the backward reads these outputs through the library: saved here,
            # autograd refuses the backward if they were modified in place
            ctx.save_for_backward(out["image"], out["final_T"])
            return out["image"], out["final_T"]

        @staticmethod
        def backward(ctx, g_image, g_T):
            image, _final_T = ctx.saved_tensors   # raises if either was modified in place
            if ctx.renderer.generation != ctx.generation:
                raise RuntimeError("the renderer rendered again before this backward")
            g_image = torch.zeros_like(image) if g_image is None else g_image
            grads = ctx.renderer.backward(ctx.scene, [g_image], [g_T] if g_T is not None else None)
            return (None, None, None, None, None, grads["means"], grads["log_scales"], grads["quats"],
                    grads["opacity_logits"], grads["sh"])

    return RenderFunction


class _LazyFunction:
    _fn = None

    def apply(self, *args):
        if _LazyFunction._fn is None:
            _LazyFunction._fn = _autograd_function()
        return _LazyFunction._fn.apply(*args)


_RenderFunction = _LazyFunction()
