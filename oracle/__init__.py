"""FP64 CPU oracle for the Gaussian-splatting forward render.

TEST INFRASTRUCTURE ONLY: ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_2607_15951_amd``) never imports this package.

The arithmetic lives in ``gs_oracle.c`` (plain C, double precision, no FMA
contraction); this module marshals numpy arrays through ctypes and strings the
steps together in the paper's order (Sec. 3.1): cull + project, bin into
(tile, depth) keys, sort, composite front to back (Eq. 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
TILE = 16

# Decision margins are reported in units of a float32 error bound (see
# composite_pixel in gs_oracle.c): below 1, a float32 evaluation of the same
# step may take the other branch of the alpha or the termination test.
ALPHA_MARGIN = 1.0
T_MARGIN = 1.0


def build(force: bool = True) -> str:
    """Compile ``gs_oracle.c`` into ``liboracle.so`` (gcc, host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11",
                               "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_p = C.c_void_p
_i64 = C.c_int64
_int = C.c_int


def _declare(L):
    L.or_sh_basis.argtypes = [_p, _p]
    L.or_debug_geometry.argtypes = [_p, _int, _int, _p, _p, _p, _p]
    L.or_debug_geometry.restype = _int
    L.or_project.argtypes = [_i64, _int, _p, _p, _p, _p, _p, _p, _int, _int] + [_p] * 10
    L.or_project.restype = _i64
    L.or_emit_pairs.argtypes = [_i64, _p, _p, _p, _int, _p, _p, _p]
    L.or_emit_pairs.restype = _i64
    L.or_sort_pairs.argtypes = [_i64, _p, _p]
    L.or_tile_ranges.argtypes = [_i64, _p, _i64, _p]
    L.or_tile_counts.argtypes = [_i64, _p, _p, _int, _i64, _p]
    L.or_tile_list.argtypes = [_i64, _p, _p, _p, _int, _i64, _p, _i64]
    L.or_tile_list.restype = _i64
    L.or_composite.argtypes = [_int, _int, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p]
    L.or_composite_pixels.argtypes = [_i64, _p, _p, _p, _i64, _i64, _p, _p, _p, _p, _p, _p, _p]
    L.or_bruteforce.argtypes = [_int, _int, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
    L.or_render_tiles.argtypes = [_int, _int, _i64] + [_p] * 8 + [_p, _i64, _p, _p, _p, _p]
    L.or_max_threads.restype = _int
    L.or_set_threads.argtypes = [_int]
    L.or_set_threads.restype = None


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def camera_array(cam: dict) -> np.ndarray:
    """R[9], t[3], fx, fy, cx, cy, near as float32 (what the render consumes)."""
    return np.concatenate([np.asarray(cam["R"], np.float32).reshape(9),
                           np.asarray(cam["t"], np.float32).reshape(3),
                           np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["near"]],
                                    np.float32)]).astype(np.float32)


def max_threads() -> int:
    return int(lib().or_max_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (<= 0: default)."""
    lib().or_set_threads(int(n))


def sh_basis(d) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(16)
    lib().or_sh_basis(_ptr(d), _ptr(out))
    return out


def debug_geometry(cam: dict, mu, log_scale, quat) -> dict | None:
    """Intermediates of one Gaussian's projection; None if culled."""
    out = np.zeros(47)
    c = camera_array(cam)
    ok = lib().or_debug_geometry(_ptr(c), int(cam["width"]), int(cam["height"]),
                                 _ptr(np.ascontiguousarray(mu, np.float64)),
                                 _ptr(np.ascontiguousarray(log_scale, np.float64)),
                                 _ptr(np.ascontiguousarray(quat, np.float64)), _ptr(out))
    o = out
    res = dict(tcam=o[0:3], Rq=o[3:12].reshape(3, 3), Sigma=o[12:21].reshape(3, 3),
               V=o[21:30].reshape(3, 3), J=o[30:36].reshape(2, 3), cov2d=o[36:39],
               conic=o[39:42], lambda_max=o[42], radius3=o[43], radius=int(o[44]),
               u=o[45], v=o[46])
    return res if ok else None


def project(scene: dict, cam: dict) -> dict:
    """Per-Gaussian projection; see ``or_project`` for the outputs."""
    n = scene["means"].shape[1]
    deg = int(scene["sh_degree"])
    W, H = int(cam["width"]), int(cam["height"])
    out = dict(mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
               rgb=np.zeros((3, n)), depth=np.zeros(n), depth_bits=np.zeros(n, np.uint32),
               radius=np.zeros(n, np.int32), rect=np.zeros((4, n), np.int32),
               tiles_touched=np.zeros(n, np.uint32), radius_margin=np.zeros(n))
    f = lambda k: np.ascontiguousarray(scene[k], np.float32)
    c = camera_array(cam)
    vis = lib().or_project(n, deg, _ptr(f("means")), _ptr(f("log_scales")), _ptr(f("quats")),
                           _ptr(f("opacity_logits")), _ptr(f("sh")), _ptr(c), W, H,
                           *[_ptr(out[k]) for k in ("mean2d", "conic", "opacity", "rgb", "depth",
                                                   "depth_bits", "radius", "rect",
                                                   "tiles_touched", "radius_margin")])
    out.update(n=n, visible=int(vis), width=W, height=H,
               tiles_x=(W + TILE - 1) // TILE, tiles_y=(H + TILE - 1) // TILE)
    return out


def bin_pairs(proj: dict):
    """Emission-order pairs: (offsets[n], keys[K], values[K])."""
    n = proj["n"]
    K = int(proj["tiles_touched"].astype(np.uint64).sum())
    offsets = np.zeros(n, np.uint64)
    keys = np.zeros(max(K, 1), np.uint64)
    values = np.zeros(max(K, 1), np.uint32)
    k2 = lib().or_emit_pairs(n, _ptr(proj["rect"]), _ptr(proj["tiles_touched"]),
                             _ptr(proj["depth_bits"]), proj["tiles_x"], _ptr(offsets),
                             _ptr(keys), _ptr(values))
    assert k2 == K
    return offsets, keys[:K], values[:K]


def sort_pairs(keys: np.ndarray, values: np.ndarray):
    keys = keys.copy()
    values = values.copy()
    lib().or_sort_pairs(len(keys), _ptr(keys), _ptr(values))
    return keys, values


def tile_ranges(keys: np.ndarray, num_tiles: int) -> np.ndarray:
    ranges = np.zeros((num_tiles, 2), np.uint64)
    lib().or_tile_ranges(len(keys), _ptr(keys), num_tiles, _ptr(ranges))
    return ranges


def tile_counts(proj: dict) -> np.ndarray:
    T = proj["tiles_x"] * proj["tiles_y"]
    counts = np.zeros(T, np.uint64)
    lib().or_tile_counts(proj["n"], _ptr(proj["rect"]), _ptr(proj["tiles_touched"]),
                         proj["tiles_x"], T, _ptr(counts))
    return counts


def tile_list(proj: dict, tile: int, cap: int | None = None) -> np.ndarray:
    """Sorted Gaussian indices of one tile, computed from the rectangles."""
    if cap is None:
        cap = 1 << 16
    while True:
        out = np.zeros(cap, np.uint32)
        m = lib().or_tile_list(proj["n"], _ptr(proj["rect"]), _ptr(proj["tiles_touched"]),
                               _ptr(proj["depth_bits"]), proj["tiles_x"], int(tile), _ptr(out), cap)
        if m <= cap:
            return out[:m]
        cap = int(m)


def composite(proj: dict, ranges: np.ndarray, values: np.ndarray, background=(0.0, 0.0, 0.0)) -> dict:
    W, H, n = proj["width"], proj["height"], proj["n"]
    P = W * H
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    margin = np.zeros((2, H, W))
    bg = np.asarray(background, np.float64)
    values = np.ascontiguousarray(values, np.uint32)
    if values.size == 0:
        values = np.zeros(1, np.uint32)
    lib().or_composite(W, H, _ptr(np.ascontiguousarray(ranges, np.uint64)), _ptr(values), n,
                       _ptr(proj["mean2d"]), _ptr(proj["conic"]), _ptr(proj["opacity"]),
                       _ptr(proj["rgb"]), _ptr(bg), _ptr(img), _ptr(T), _ptr(nc), _ptr(margin))
    del P
    return dict(image=img, final_T=T, n_contrib=nc, margin_alpha=margin[0], margin_T=margin[1])


def composite_pixels(proj: dict, px, py, tile_values: np.ndarray, background=(0.0, 0.0, 0.0)):
    """Composite selected pixels of one tile along that tile's sorted list.

    Returns (out[k, 5] = r, g, b, final T, n_contrib; margins[k, 2])."""
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    k = len(px)
    out = np.zeros((k, 5))
    marg = np.zeros((k, 2))
    vals = np.ascontiguousarray(tile_values, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
        length = 0
    else:
        length = len(tile_values)
    lib().or_composite_pixels(k, _ptr(px), _ptr(py), _ptr(vals), length, proj["n"],
                              _ptr(proj["mean2d"]), _ptr(proj["conic"]), _ptr(proj["opacity"]),
                              _ptr(proj["rgb"]), _ptr(np.asarray(background, np.float64)),
                              _ptr(out), _ptr(marg))
    return out, marg


def render_tiles(proj: dict, tiles=None, background=(0.0, 0.0, 0.0), out: dict | None = None) -> dict:
    """The given tiles (row-major indices; all when None), each from its own
    list and composited pixel by pixel, without emitting or sorting every
    pair of the frame: the same lists and per-pixel walk as ``render``, for
    whole large frames or for the tiles a change touches.  Writes only those
    tiles' pixels of ``out`` (new zero arrays when None) and returns it."""
    W, H, n = proj["width"], proj["height"], proj["n"]
    T = proj["tiles_x"] * proj["tiles_y"]
    tl = np.arange(T, dtype=np.int64) if tiles is None else np.ascontiguousarray(tiles, np.int64)
    if out is None:
        out = dict(image=np.zeros((3, H, W)), final_T=np.zeros((H, W)), n_contrib=np.zeros((H, W), np.int32),
                   margin=np.zeros((2, H, W)))
    if len(tl):
        lib().or_render_tiles(W, H, n, _ptr(proj["rect"]), _ptr(proj["tiles_touched"]), _ptr(proj["depth_bits"]),
                              _ptr(proj["mean2d"]), _ptr(proj["conic"]), _ptr(proj["opacity"]), _ptr(proj["rgb"]),
                              _ptr(np.asarray(background, np.float64)), _ptr(tl), len(tl), _ptr(out["image"]),
                              _ptr(out["final_T"]), _ptr(out["n_contrib"]), _ptr(out["margin"]))
    out["margin_alpha"], out["margin_T"] = out["margin"][0], out["margin"][1]
    return out


def bruteforce(proj: dict, background=(0.0, 0.0, 0.0)) -> dict:
    """Every pixel composites every geometrically valid Gaussian (no tiles)."""
    W, H, n = proj["width"], proj["height"], proj["n"]
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    lib().or_bruteforce(W, H, n, _ptr(proj["radius_margin"]), _ptr(proj["depth"]),
                        _ptr(proj["mean2d"]), _ptr(proj["conic"]), _ptr(proj["opacity"]),
                        _ptr(proj["rgb"]), _ptr(np.asarray(background, np.float64)),
                        _ptr(img), _ptr(T), _ptr(nc))
    return dict(image=img, final_T=T, n_contrib=nc)


def render(scene: dict, cam: dict, background=(0.0, 0.0, 0.0)) -> dict:
    """The whole forward path: project, bin, sort, ranges, composite."""
    proj = project(scene, cam)
    offsets, keys, values = bin_pairs(proj)
    skeys, svals = sort_pairs(keys, values)
    T = proj["tiles_x"] * proj["tiles_y"]
    ranges = tile_ranges(skeys, T)
    comp = composite(proj, ranges, svals, background)
    return dict(proj=proj, offsets=offsets, keys=skeys, values=svals, ranges=ranges, **comp)


def ambiguous_mask(res: dict, alpha_margin: float = ALPHA_MARGIN, t_margin: float = T_MARGIN):
    """Pixels whose threshold decisions sit within float32 reach of the edge."""
    return (res["margin_alpha"] < alpha_margin) | (res["margin_T"] < t_margin)
