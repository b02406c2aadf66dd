"""Seeded synthetic scenes and cameras for the Gaussian-splatting render path.

This module only draws random numbers and lays them out; it holds none of the
rendering arithmetic.  Both the FP64 oracle (``oracle/``) and the HIP library
consume the arrays it returns, so it is the single source of inputs for parity
tests, ``bench.py`` and ``__graft_entry__.smoke()``.

Layout (structure of arrays, channel-major, float32):

* ``means``          ``[3, N]``   world-space centres
* ``log_scales``     ``[3, N]``   per-axis log standard deviations
* ``quats``          ``[4, N]``   rotation quaternion ``(w, x, y, z)``
* ``opacity_logits`` ``[N]``      opacity before the sigmoid
* ``sh``             ``[(L+1)^2, 3, N]``  spherical-harmonic coefficients,
  coefficient-major, then colour channel

The scene parameterisation (mean, rotation + scale covariance, opacity, SH
colour) follows the background section on 3D Gaussian Splatting (Sec. 3.1);
the Gaussian record of Sec. 4.5 (Gaussian representation) stores the same fields with log-space scale.

The paper measures on SLAM-exported scenes that are not available here; the
five workloads below stand in for them (see ``CONFIGS``).
"""
from __future__ import annotations

import math

import numpy as np

# Y_0^0 of the real SH basis, 1 / (2 sqrt(pi)); used only to turn a drawn RGB
# value into the DC coefficient that reproduces it (a layout detail of the
# input, not part of the render arithmetic).
_Y00 = 0.5 / math.sqrt(math.pi)

CONFIGS = {
    "C1": dict(kind="uniform", n=1_000, width=128, height=128, sh_degree=0, seed=1),
    "C2": dict(kind="mixture", n=500_000, width=1280, height=720, sh_degree=3, seed=2,
               components=64),
    "C3": dict(kind="powerlaw", n=3_000_000, width=1920, height=1080, sh_degree=3, seed=3),
    "C4": dict(kind="mixture", n=1_000_000, width=0, height=0, sh_degree=3, seed=4,
               components=64, cameras=64),
    "C5": dict(kind="powerlaw", n=6_000_000, width=3840, height=2160, sh_degree=3, seed=5),
}

WORKLOAD_NAMES = {
    "C1": "plain forward fp32, 1k Gaussians uniform in [-1,1]^3, SH0, 128x128",
    "C2": "forward fp32, 500k Gaussians, 64-component mixture, SH3, 1280x720",
    "C3": "forward fp32, 3M Gaussians, 256-cluster power-law mixture + 10% background, SH3, 1920x1080",
    "C4": "batched, 1M-Gaussian mixture, SH3, 64 cameras of mixed resolution",
    "C5": "precision variant, 6M Gaussians power-law mixture + background, SH3, 3840x2160",
}


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree):
    rgb = rng.uniform(0.0, 1.0, (3, n))
    coeffs = np.empty(((degree + 1) ** 2, 3, n))
    coeffs[0] = (rgb - 0.5) / _Y00
    if degree > 0:
        coeffs[1:] = rng.normal(0.0, 0.2, ((degree + 1) ** 2 - 1, 3, n))
    return coeffs


def _mixture_means(rng, n, components):
    centres = rng.uniform(-1.0, 1.0, (components, 3))
    stds = np.exp(rng.uniform(math.log(0.05), math.log(0.25), components))
    weights = rng.dirichlet(np.ones(components))
    comp = rng.choice(components, size=n, p=weights)
    offs = rng.standard_normal((n, 3))
    return (centres[comp] + stds[comp, None] * offs).T


def _largest_remainder(total, weights):
    share = total * weights / weights.sum()
    base = np.floor(share).astype(np.int64)
    rest = total - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rest]] += 1
    return base


def _powerlaw_means(rng, n_fg, n_bg, clusters=256):
    draws = rng.pareto(1.5, clusters) + 1.0           # classical Pareto(a=1.5), x_m = 1
    sizes = _largest_remainder(n_fg, draws)
    centres = rng.uniform(-1.0, 1.0, (clusters, 3))
    stds = np.exp(rng.uniform(math.log(0.02), math.log(0.2), clusters))
    comp = np.repeat(np.arange(clusters), sizes)
    fg = centres[comp] + stds[comp, None] * rng.standard_normal((n_fg, 3))
    dirs = rng.standard_normal((n_bg, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    radii = rng.uniform(8.0, 12.0, n_bg)
    bg = dirs * radii[:, None]
    return np.concatenate([fg, bg]).T


def make_scene(config: str, n: int | None = None, seed: int | None = None,
               sh_degree: int | None = None) -> dict:
    """Draw the Gaussians of workload ``config`` ("C1".."C5").

    ``n``, ``seed`` and ``sh_degree`` override the workload's values (used for
    small parity cases that keep a workload's distribution).  Draw order is
    fixed: means, log-scales, quaternions, logits, SH, then (power-law scenes
    only) a random permutation of the Gaussian order, so that index order
    carries no spatial structure.
    """
    cfg = dict(CONFIGS[config])
    n = cfg["n"] if n is None else int(n)
    seed = cfg["seed"] if seed is None else int(seed)
    deg = cfg["sh_degree"] if sh_degree is None else int(sh_degree)
    rng = np.random.default_rng(seed)
    kind = cfg["kind"]
    if kind == "uniform":
        means = rng.uniform(-1.0, 1.0, (3, n))
        log_scales = rng.normal(-3.0, 0.5, (3, n))
    elif kind == "mixture":
        means = _mixture_means(rng, n, cfg["components"])
        log_scales = rng.normal(-4.0, 0.7, (3, n))
    elif kind == "powerlaw":
        n_bg = n // 10
        n_fg = n - n_bg
        means = _powerlaw_means(rng, n_fg, n_bg)
        log_scales = np.concatenate([rng.normal(-4.0, 0.7, (3, n_fg)),
                                     rng.normal(-1.0, 0.5, (3, n_bg))], axis=1)
    else:
        raise ValueError(kind)
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = _sh(rng, n, deg)
    if kind == "powerlaw":
        perm = rng.permutation(n)
        means, log_scales, quats = means[:, perm], log_scales[:, perm], quats[:, perm]
        logits, sh = logits[perm], sh[..., perm]
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(means=f32(means), log_scales=f32(log_scales), quats=f32(quats),
                opacity_logits=f32(logits), sh=f32(sh), sh_degree=deg)


def default_camera(width: int, height: int, fov_deg: float = 60.0) -> dict:
    """Pinhole camera at world (0, 0, -3) looking down +z (x right, y down).

    ``R``/``t`` map world to camera coordinates; f = (W/2)/tan(fov/2) on both
    axes, principal point (W/2, H/2); near plane 0.2.
    """
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return dict(R=np.eye(3, dtype=np.float32), t=np.array([0.0, 0.0, 3.0], np.float32),
                fx=np.float32(f), fy=np.float32(f), cx=np.float32(width / 2.0),
                cy=np.float32(height / 2.0), near=np.float32(0.2),
                width=int(width), height=int(height))


def look_at_camera(eye, width: int, height: int, fov_deg: float = 60.0) -> dict:
    """Camera at ``eye`` looking at the origin, image y along world +y (down)."""
    eye = np.asarray(eye, np.float64)
    fwd = -eye / np.linalg.norm(eye)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, fwd)
    if np.linalg.norm(right) < 1e-6:
        down = np.array([0.0, 0.0, 1.0])
        right = np.cross(down, fwd)
    right /= np.linalg.norm(right)
    down_c = np.cross(fwd, right)
    R = np.stack([right, down_c, fwd])
    t = -R @ eye
    cam = default_camera(width, height, fov_deg)
    cam["R"] = R.astype(np.float32)
    cam["t"] = t.astype(np.float32)
    return cam


def make_cameras(config: str) -> list[dict]:
    """Cameras of a workload: one default camera, or (C4) 64 look-at cameras.

    C4: eyes at 4 * normalise(N(0, I3)), resolutions drawn uniformly from
    {256x256, 640x480, 1280x720, 1920x1080}; seed = workload seed + 1000.
    """
    cfg = CONFIGS[config]
    if cfg.get("cameras"):
        rng = np.random.default_rng(cfg["seed"] + 1000)
        sizes = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]
        cams = []
        for _ in range(cfg["cameras"]):
            e = rng.standard_normal(3)
            e = 4.0 * e / np.linalg.norm(e)
            w, h = sizes[int(rng.integers(0, 4))]
            cams.append(look_at_camera(e, w, h))
        return cams
    return [default_camera(cfg["width"], cfg["height"])]


def ring_cameras(count: int, width: int, height: int, radius: float = 3.0) -> list[dict]:
    """``count`` look-at cameras evenly spaced on a circle of ``radius`` in the
    xz-plane around the origin (the batched form of the C3 workload uses 8 at
    1920x1080); the first sits at (0, 0, -radius), the default camera's eye."""
    cams = []
    for k in range(count):
        a = 2.0 * math.pi * k / count
        cams.append(look_at_camera((radius * math.sin(a), 0.0, -radius * math.cos(a)), width, height))
    return cams


def orbit_camera(angle_deg: float, width: int, height: int, radius: float = 3.0) -> dict:
    """Look-at camera on the same circle as ring_cameras at ``angle_deg``
    degrees (0 = the default camera's eye): frames of an orbit, as in the
    churn measurements of Sec. 5.7 (Table 5)."""
    a = math.radians(angle_deg)
    return look_at_camera((radius * math.sin(a), 0.0, -radius * math.cos(a)), width, height)


def random_target(width: int, height: int, seed: int = 33) -> np.ndarray:
    """Uniform [0,1) target image ``[3, H, W]`` for an L2 loss."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, (3, height, width)).astype(np.float32)


def to_bf16_storage(a: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round-to-nearest-even); returns uint16 bits."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((b >> 16) & 1) + 0x7FFF
    return ((b + rounding) >> 16).astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)
