"""FP64 differentiable twin of the oracle's render, for gradients.

TEST INFRASTRUCTURE ONLY (as the rest of ``oracle/``): only ``tests/`` use it.

The forward follows the same steps and readings as ``gs_oracle.c`` (Sec. 3.1
stages 1, 2 and 4; Eq. 1), written with plain PyTorch CPU operations in
float64 so that ``torch.autograd`` gives the gradient of a loss of the image
with respect to the Gaussian parameters.  The discrete parts -- which
Gaussians are visible, their tile rectangles and every tile's depth-sorted
list -- come from the C oracle and are held fixed, as in the method (the
sort order is piecewise constant).  The alpha threshold (skip a < 1/255),
the 0.99 clamp and the early termination are applied as masks computed from
the values; they pass no gradient.

Pinned in ``tests/test_oracle_grad.py``: its forward equals the C oracle's
image and final transmittance, and its gradient equals central finite
differences of the C oracle's render.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import camera_array, project, tile_list

TILE = 16
_PI = math.pi


def sh_basis_t(x, y, z, degree: int):
    """Real SH basis (Condon-Shortley phase, index l*l + l + m) of unit
    directions, as in or_sh_basis; list of tensors."""
    out = [torch.full_like(x, 0.5 * math.sqrt(1.0 / _PI))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * _PI))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        out += [0.5 * math.sqrt(15.0 / _PI) * x * y, -0.5 * math.sqrt(15.0 / _PI) * y * z,
                0.25 * math.sqrt(5.0 / _PI) * (3.0 * z * z - 1.0), -0.5 * math.sqrt(15.0 / _PI) * x * z,
                0.25 * math.sqrt(15.0 / _PI) * (x * x - y * y)]
    if degree >= 3:
        out += [-0.25 * math.sqrt(35.0 / (2.0 * _PI)) * y * (3.0 * x * x - y * y),
                0.5 * math.sqrt(105.0 / _PI) * x * y * z,
                -0.25 * math.sqrt(21.0 / (2.0 * _PI)) * y * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(7.0 / _PI) * z * (5.0 * z * z - 3.0),
                -0.25 * math.sqrt(21.0 / (2.0 * _PI)) * x * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(105.0 / _PI) * z * (x * x - y * y),
                -0.25 * math.sqrt(35.0 / (2.0 * _PI)) * x * (x * x - 3.0 * y * y)]
    return out


def project_t(params: dict, cam: dict, idx: torch.Tensor):
    """Differentiable projection of the Gaussians ``idx`` (all visible):
    centre (u, v), conic (A, B, C), opacity, rgb [3]."""
    mu = params["means"][:, idx]
    ls = params["log_scales"][:, idx]
    q = params["quats"][:, idx]
    c = camera_array(cam).astype(np.float64)    # the float32 camera the render reads
    W = torch.as_tensor(c[0:9].reshape(3, 3))
    tc = torch.as_tensor(c[9:12])
    fx, fy, cx, cy = (float(x) for x in c[12:16])
    W_img, H_img = int(cam["width"]), int(cam["height"])
    t = W @ mu + tc[:, None]
    qn = q / torch.sqrt((q * q).sum(0, keepdim=True))
    w, x, y, z = qn
    R = torch.stack([torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
                     torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
                     torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])
    R = R.permute(2, 0, 1)                                  # [m, 3, 3]
    M = R * torch.exp(ls).T[:, None, :]                     # R diag(s)
    Sigma = M @ M.transpose(1, 2)
    V = W[None] @ Sigma @ W.T[None]
    tx, ty, tz = t
    limx = 1.3 * (0.5 * W_img / fx)
    limy = 1.3 * (0.5 * H_img / fy)
    xcl = torch.clamp(tx / tz, -limx, limx) * tz
    ycl = torch.clamp(ty / tz, -limy, limy) * tz
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * xcl / (tz * tz)]),
                     torch.stack([zero, fy / tz, -fy * ycl / (tz * tz)])]).permute(2, 0, 1)   # [m, 2, 3]
    P = J @ V @ J.transpose(1, 2)
    a = P[:, 0, 0] + 0.3
    b = P[:, 0, 1]
    c = P[:, 1, 1] + 0.3
    det = a * c - b * b
    A, B, Cc = c / det, -b / det, a / det
    u = fx * tx / tz + cx
    v = fy * ty / tz + cy
    opacity = torch.sigmoid(params["opacity_logits"][idx])
    # view-dependent colour
    campos = -(W.T @ tc)
    d = mu - campos[:, None]
    d = d / torch.sqrt((d * d).sum(0, keepdim=True))
    deg = int(params["sh_degree"])
    Y = sh_basis_t(d[0], d[1], d[2], deg)
    sh = params["sh"][:, :, idx]                            # [ncoef, 3, m]
    rgb = sum(sh[k] * Y[k][None] for k in range(len(Y))) + 0.5
    rgb = torch.clamp(rgb, min=0.0)
    return u, v, A, B, Cc, opacity, rgb


def composite_tile_t(u, v, A, B, Cc, op, rgb, px, py, bg):
    """Eq. 1 front to back for pixels (px, py) along one tile list (already
    restricted to the list's Gaussians in order); returns colour [3, P],
    final transmittance [P] and the composited mask [P, len]."""
    dx = u[None, :] - px[:, None]
    dy = v[None, :] - py[:, None]
    power = -0.5 * (A[None] * dx * dx + Cc[None] * dy * dy) - B[None] * dx * dy
    raw = op[None] * torch.exp(power)
    alpha = torch.clamp(raw, max=0.99)
    with torch.no_grad():
        include = alpha >= 1.0 / 255.0
        one_minus = torch.where(include, 1.0 - alpha, torch.ones_like(alpha))
        T_excl = torch.cumprod(torch.cat([torch.ones_like(one_minus[:, :1]), one_minus[:, :-1]], 1), 1)
        stop = include & (T_excl * (1.0 - alpha) < 1e-4)
        after = torch.cumsum(stop.to(torch.int64), 1) > 0   # from the first stop on
        keep = include & ~after
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    one = 1.0 - a
    T = torch.cumprod(torch.cat([torch.ones_like(one[:, :1]), one[:, :-1]], 1), 1)
    w = a * T
    colour = (w[None] * rgb[:, None, :]).sum(-1)           # [3, P]
    Tf = torch.prod(one, 1)
    bg = torch.as_tensor(np.asarray(bg, np.float64))
    return colour + Tf[None] * bg[:, None], Tf, keep


def render_t(params: dict, cam: dict, background=(0.0, 0.0, 0.0), tiles=None, proj=None):
    """Differentiable FP64 render of the tiles ``tiles`` (all when None).

    ``params`` holds float64 tensors means [3,N], log_scales [3,N], quats
    [4,N], opacity_logits [N], sh [(L+1)^2,3,N] and sh_degree; the visible
    set, rectangles and tile lists come from the C oracle's projection of the
    same values (``proj``, computed when None).  Returns {tile: (px, py,
    colour [3,P], final_T [P], composited mask [P, len])}."""
    if proj is None:
        scene = {k: (params[k].detach().numpy().astype(np.float32) if k != "sh_degree" else params[k])
                 for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "sh_degree")}
        proj = project(scene, cam)
    W, H = int(cam["width"]), int(cam["height"])
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    if tiles is None:
        tiles = range(tx * ty)
    out = {}
    for t in tiles:
        lst = tile_list(proj, int(t)).astype(np.int64)
        x0, y0 = (t % tx) * TILE, (t // tx) * TILE
        ys, xs = np.mgrid[y0:min(y0 + TILE, H), x0:min(x0 + TILE, W)]
        px = torch.as_tensor(xs.ravel().astype(np.float64))
        py = torch.as_tensor(ys.ravel().astype(np.float64))
        if len(lst) == 0:
            bg = torch.as_tensor(np.asarray(background, np.float64))
            out[int(t)] = (xs.ravel(), ys.ravel(), bg[:, None].expand(3, len(px)).clone(),
                           torch.ones(len(px), dtype=torch.float64), torch.zeros((len(px), 0), dtype=torch.bool))
            continue
        idx = torch.as_tensor(lst)
        u, v, A, B, Cc, op, rgb = project_t(params, cam, idx)
        colour, Tf, keep = composite_tile_t(u, v, A, B, Cc, op, rgb, px, py, background)
        out[int(t)] = (xs.ravel(), ys.ravel(), colour, Tf, keep)
    return out


def image_t(params: dict, cam: dict, background=(0.0, 0.0, 0.0), proj=None):
    """The whole image [3, H, W] and final transmittance [H, W] as tensors."""
    W, H = int(cam["width"]), int(cam["height"])
    img = torch.zeros((3, H, W), dtype=torch.float64)
    Tf = torch.zeros((H, W), dtype=torch.float64)
    parts = render_t(params, cam, background, proj=proj)
    for t, (xs, ys, colour, T, _) in parts.items():
        img = img.index_put((torch.arange(3)[:, None], torch.as_tensor(ys)[None], torch.as_tensor(xs)[None]), colour)
        Tf = Tf.index_put((torch.as_tensor(ys), torch.as_tensor(xs)), T)
    return img, Tf


def loss_t(params: dict, cam: dict, w_rgb, w_T, background=(0.0, 0.0, 0.0), tiles=None, proj=None):
    """L = sum(w_rgb * image) + sum(w_T * final_T) over the tiles ``tiles``
    (numpy weights [3,H,W] and [H,W]); also returns the composited masks."""
    parts = render_t(params, cam, background, tiles=tiles, proj=proj)
    L = torch.zeros((), dtype=torch.float64)
    masks = {}
    for t, (xs, ys, colour, T, keep) in parts.items():
        wr = torch.as_tensor(np.asarray(w_rgb, np.float64)[:, ys, xs])
        wt = torch.as_tensor(np.asarray(w_T, np.float64)[ys, xs])
        L = L + (wr * colour).sum() + (wt * T).sum()
        masks[t] = keep
    return L, masks


def gradients(params: dict, cam: dict, w_rgb, w_T, background=(0.0, 0.0, 0.0), tiles=None, proj=None) -> dict:
    """dL/d(parameter) of ``loss_t`` as float64 numpy arrays."""
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        if params[k].grad is not None:
            params[k].grad = None
    L, _ = loss_t(params, cam, w_rgb, w_T, background, tiles=tiles, proj=proj)
    L.backward()
    return {k: (params[k].grad.numpy().copy() if params[k].grad is not None else np.zeros(params[k].shape))
            for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}


def params_from_scene(scene: dict, requires_grad: bool = True) -> dict:
    """float64 leaf tensors of a scene's float32 arrays."""
    p = {k: torch.tensor(np.asarray(scene[k], np.float64), requires_grad=requires_grad)
         for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    p["sh_degree"] = int(scene["sh_degree"])
    return p
