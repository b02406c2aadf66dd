"""Finite-difference check of the backward on the full bench workload: 3M
Gaussians, SH3, 1920x1080, loss = L2 to a seeded random target image.

The GPU gradient (gs_render_backward through Renderer.backward) of sampled
parameters of 20 seen Gaussians (the frontmost of seeded tiles' lists) is
compared with central differences of the FP64 oracle's loss.
The oracle re-renders only the tiles of the perturbed Gaussian's 3-sigma
rectangle (oracle.render_tiles builds each tile's list from scratch, so a
changed depth order is taken into account), with the rest of the projection
held at the base values.  The loss weight is zero on pixels whose compositing
decisions the oracle marks ambiguous (there the float32 render may take the
other branch) and outside the sampled Gaussians' tiles.

The backward holds the rectangles and the depth order fixed and passes no
gradient through the 1/255 skip, the 0.99 clamp or termination: the
differences keep the perturbed Gaussian's depth key (its list positions) at
the rendered value, and a sample whose perturbation changes its rectangle, or
whose differences at h and h/2 disagree (a decision flipped inside the step),
is not smooth there and is redrawn.
"""
import json
import sys

import numpy as np
import pytest

import oracle
import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

TILE = 16
N_GAUSSIANS = 20
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
# relative step per parameter group (of max(|value|, floor)): small, since
# the number of pixels whose 1/255 alpha test flips inside the step grows with
# it (such a sample is redrawn), yet hundreds of float32 ulps of the value
# (the effective step is taken from the rounded values), with FP64 roundoff
# of the loss difference near 1e-7
STEP = {"means": (2e-6, 1.0), "log_scales": (1e-4, 1.0), "quats": (1e-4, 1.0), "opacity_logits": (1e-4, 1.0),
        "sh": (1e-4, 0.2)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def renderer():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_15951_amd as gs
    r = gs.Renderer(0)
    yield r
    r.close()


def rect_tiles(rect, tiles_x):
    x0, y0, x1, y1 = (int(v) for v in rect)
    return np.array([ty * tiles_x + tx for ty in range(y0, y1) for tx in range(x0, x1)], np.int64)


def tile_mask(tiles, tiles_x, W, H):
    m = np.zeros((H, W), bool)
    for t in tiles:
        x0, y0 = (t % tiles_x) * TILE, (t // tiles_x) * TILE
        m[y0:y0 + TILE, x0:x0 + TILE] = True
    return m


def param_view(scene, group, i, k):
    """(array, index) of parameter k of Gaussian i in its group."""
    a = scene[group]
    if group == "opacity_logits":
        return a, (i,)
    if group == "sh":
        return a, (k // 3, k % 3, i)
    return a, (k, i)


def test_c3_gradients_against_finite_differences(renderer):
    import torch
    import paper_2607_15951_amd as gs
    scene = scenes.make_scene("C3")
    cam = scenes.make_cameras("C3")[0]
    W, H = cam["width"], cam["height"]
    n = scene["means"].shape[1]
    target = scenes.random_target(W, H, seed=33)
    base = oracle.project(scene, cam)
    tx = base["tiles_x"]
    # the sampled Gaussians: in each of a seeded sequence of tiles, the
    # frontmost entry of the tile's list whose rectangle spans at most 300
    # tiles (each difference re-renders them four times) and that lies before
    # the tile's largest n_contrib, so that pixels composite it.  (A seeded
    # subset of all Gaussians would be almost all hidden: a pixel of this
    # dense scene terminates after about 3% of its tile's list.)
    ntiles = (base["rect"][2] - base["rect"][0]) * (base["rect"][3] - base["rect"][1])
    rng = np.random.default_rng(303)
    picks = []
    for t in rng.permutation(base["tiles_x"] * base["tiles_y"]):
        lst = oracle.tile_list(base, int(t))
        nc = int(oracle.render_tiles(base, [int(t)])["n_contrib"].max())
        for pos in range(min(nc, len(lst))):
            i = int(lst[pos])
            if ntiles[i] <= 300 and i not in picks:
                picks.append(i)
                break
        if len(picks) == N_GAUSSIANS:
            break
    union = np.unique(np.concatenate([rect_tiles(base["rect"][:, i], tx) for i in picks]))
    say(f"[fd] {len(picks)} Gaussians sampled over {len(union)} tiles")
    b = oracle.render_tiles(base, union)
    keep = tile_mask(union, tx, W, H) & ~oracle.ambiguous_mask(b)

    # GPU gradient of L = sum(w (img - target)^2)
    dev = gs.scene_to_device(scene)
    out = renderer.render(dev, cam, W, H)
    torch.cuda.synchronize()
    img = out["image"].cpu().numpy().astype(np.float64)
    g_img = 2.0 * keep[None] * (img - target)
    grads = renderer.backward(dev, [torch.from_numpy(g_img.astype(np.float32)).cuda()])
    torch.cuda.synchronize()
    grads = {k: v.cpu().numpy() for k, v in grads.items()}
    # the GPU image agrees with the oracle's on the kept pixels (parity)
    assert float(np.abs(img - b["image"])[:, keep].max()) <= 1e-4

    def loss_on(proj, tiles):
        r = oracle.render_tiles(proj, tiles)
        m = tile_mask(tiles, tx, W, H) & keep
        return float((((r["image"] - target) ** 2) * m[None]).sum())

    work = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    fields = ("mean2d", "conic", "opacity", "rgb", "depth", "depth_bits", "radius", "rect", "tiles_touched",
              "radius_margin")
    results, redrawn = [], 0
    for i in picks:
        tiles = rect_tiles(base["rect"][:, i], tx)
        for group in GROUPS:
            count = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "sh": 48}[group]
            order = list(rng.permutation(count))
            done = False
            while order and not done:
                k = int(order.pop())
                arr, idx = param_view(work, group, i, k)
                x0 = float(arr[idx])
                rel, floor = STEP[group]
                fd = {}
                ok = True
                for h in (rel * max(abs(x0), floor), 0.5 * rel * max(abs(x0), floor)):
                    vals = []
                    for sgn in (1.0, -1.0):
                        arr[idx] = np.float32(x0 + sgn * h)
                        one = {f: (np.ascontiguousarray(work[f][..., i:i + 1]) if isinstance(work[f], np.ndarray)
                                   else work[f]) for f in work}
                        p1 = oracle.project(one, cam)
                        if p1["tiles_touched"][0] != base["tiles_touched"][i] or \
                                not np.array_equal(p1["rect"][:, 0], base["rect"][:, i]):
                            ok = False
                        saved = {f: np.array(base[f][..., i], copy=True) for f in fields}
                        for f in fields:
                            base[f][..., i] = p1[f][..., 0]
                        # the depth order stays as rendered: the backward holds
                        # every tile list and its order fixed (the sort has no
                        # gradient), while a step in depth would pass
                        # neighbours about 1e-6 apart
                        base["depth_bits"][i] = saved["depth_bits"]
                        vals.append(loss_on(base, tiles))
                        for f in fields:
                            base[f][..., i] = saved[f]
                    h_eff = (float(np.float32(x0 + h)) - float(np.float32(x0 - h))) / 2.0
                    fd[h] = (vals[0] - vals[1]) / (2.0 * h_eff)
                    arr[idx] = np.float32(x0)
                    if not ok:
                        break
                if not ok:
                    redrawn += 1
                    continue
                f_big, f_small = fd.values()
                scale = max(abs(f_small), 1e-6)
                if abs(f_big - f_small) > 2e-3 * scale + 1e-7:
                    redrawn += 1   # a decision flipped inside the step
                    continue
                gi = float(grads[group][idx])
                results.append(dict(gaussian=i, group=group, k=k, fd=f_small, gpu=gi))
                done = True
    say(f"[fd] {len(results)} compared, {redrawn} redrawn")
    by_group = {}
    for r in results:
        by_group.setdefault(r["group"], []).append(r)
    worst = {}
    for group, rs in by_group.items():
        fdv = np.array([r["fd"] for r in rs])
        gpv = np.array([r["gpu"] for r in rs])
        G = float(np.abs(fdv).max())
        err = np.abs(gpv - fdv)
        # float32 recomputation in the backward (about 1e-5 of the group's
        # largest gradient) and the O(h^2) truncation of the difference
        assert G > 0, f"{group}: every sampled gradient is zero"
        assert (err <= 2e-3 * np.abs(fdv) + 2e-4 * G).all(), (group, list(zip(fdv, gpv)))
        worst[group] = float((err / (np.abs(fdv) + 2e-4 * G)).max())
        # most samples carry a gradient of their own, not only the group's largest
        assert (np.abs(fdv) > 1e-3 * G).mean() >= 0.5, (group, fdv)
    counts = {g: len(rs) for g, rs in by_group.items()}
    say("[fd] " + json.dumps({"compared": len(results), "redrawn": redrawn, "per_group": counts,
                             "worst_relative_by_group": worst}))
    # a group whose few parameters all flip a decision inside the step for a
    # Gaussian contributes nothing for it; every group still gets its share
    assert len(results) >= 45 and all(counts.get(g, 0) >= 6 for g in GROUPS), counts
