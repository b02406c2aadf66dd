"""GPU parity of the backward (gs_render_backward, the autograd wrapper)
against the FP64 autograd oracle ``oracle.grad``.

The loss is L = sum(w_rgb * image) + sum(w_T * final_T) with seeded random
weights, so dL/d(image) = w_rgb and dL/d(final_T) = w_T are what the backward
receives.  Pixels whose threshold decisions are within float32 reach of the
edge (the oracle's ambiguity margins) get zero weight on both sides: there the
two renders may composite different sets and the loss is not the same
function.  Gradients of every parameter group are compared with the oracle's
by norm-relative error and by the largest element error relative to the
group's largest gradient.
"""
import sys

import numpy as np
import pytest

import oracle
import scenes
from parity import check_projection, dequantised

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
TILE = 16
# The kernels recompute each pixel's transmittance and the colour behind an
# entry in float32 along the composited entries: both carry about 2u relative
# error per composited entry (u = 2^-24), and pixels of these scenes composite
# at most a few hundred entries, so an element's error stays below ~1e-4 of the
# largest gradient of its group; the norm-relative error averages it further.
NORM_TOL = 5e-5
MAX_TOL = 1e-4


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


def loss_weights(cam, seed, ambiguous=None, tiles=None):
    """Seeded weights in [-1, 1]; zero on ambiguous pixels and, when
    ``tiles`` is given, outside those tiles."""
    rng = np.random.default_rng(seed)
    H, W = cam["height"], cam["width"]
    w_rgb = rng.uniform(-1.0, 1.0, (3, H, W))
    w_T = rng.uniform(-1.0, 1.0, (H, W))
    keep = np.ones((H, W), bool)
    if tiles is not None:
        keep[:] = False
        tx = (W + TILE - 1) // TILE
        for t in tiles:
            x0, y0 = (t % tx) * TILE, (t // tx) * TILE
            keep[y0:y0 + TILE, x0:x0 + TILE] = True
    if ambiguous is not None:
        keep &= ~ambiguous
    return w_rgb * keep, w_T * keep


def compare(label, got: dict, want: dict, idx=None):
    errs = {}
    for k in GROUPS:
        g = np.asarray(got[k], np.float64)
        w = np.asarray(want[k], np.float64)
        if idx is not None:
            g = g[..., idx]
        assert np.all(np.isfinite(g)), f"{label} {k}: non-finite gradient"
        scale = float(np.abs(w).max())
        nrm = float(np.linalg.norm(w))
        d = g - w
        e_norm = float(np.linalg.norm(d)) / nrm if nrm > 0 else float(np.linalg.norm(d))
        e_max = float(np.abs(d).max()) / scale if scale > 0 else float(np.abs(d).max())
        errs[k] = (e_norm, e_max)
    say(f"[backward] {label}: " + " ".join(f"{k}=({a:.1e},{b:.1e})" for k, (a, b) in errs.items()))
    for k, (a, b) in errs.items():
        assert a <= NORM_TOL, f"{label} {k}: norm-relative error {a:.3e}"
        assert b <= MAX_TOL, f"{label} {k}: max error {b:.3e} of the largest gradient"


def gpu_grads(renderer, dev, w_rgb, w_T, views=1):
    import torch
    gi = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda() for w in w_rgb]
    gt = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda() for w in w_T]
    g = renderer.backward(dev, gi, gt)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


def oracle_grads(scene, cam, w_rgb, w_T, bg, proj=None, tiles=None):
    import oracle.grad as og
    p = og.params_from_scene(scene)
    return og.gradients(p, cam, w_rgb, w_T, bg, tiles=tiles, proj=proj)


def small_case(renderer, scene, cam, label, dtype=0, bg=(0.0, 0.0, 0.0), seed=1):
    import paper_2607_15951_amd as gs
    say(f"[backward] {label}: n={scene['means'].shape[1]} {cam['width']}x{cam['height']} dtype={dtype}")
    dev = gs.scene_to_device(scene, dtype)
    renderer.render(dev, cam, cam["width"], cam["height"], background=bg)
    ref_scene = dequantised(scene, dtype)
    o = oracle.render(ref_scene, cam, background=bg)
    assert o["proj"]["visible"] > 0
    w_rgb, w_T = loss_weights(cam, seed, ambiguous=oracle.ambiguous_mask(o))
    got = gpu_grads(renderer, dev, [w_rgb], [w_T])
    want = oracle_grads(ref_scene, cam, w_rgb, w_T, bg, proj=o["proj"])
    compare(label, got, want)
    return got, want


def enlarged(scene, by=1.6):
    scene = dict(scene)
    scene["log_scales"] = (scene["log_scales"] + np.float32(by)).astype(np.float32)
    return scene


def test_backward_sh0_ragged(renderer):
    sc = enlarged(scenes.make_scene("C1", n=300, seed=41, sh_degree=0))
    small_case(renderer, sc, scenes.default_camera(72, 50), "SH0 300 72x50", bg=(0.2, 0.4, 0.1), seed=3)


def test_backward_sh3_rotated(renderer):
    sc = enlarged(scenes.make_scene("C2", n=400, seed=42), by=2.2)
    cam = scenes.look_at_camera([1.1, -0.6, -2.6], 90, 70)
    small_case(renderer, sc, cam, "SH3 400 rotated 90x70", seed=4)


def test_backward_powerlaw_sh1(renderer):
    sc = scenes.make_scene("C3", n=3000, seed=43, sh_degree=1)
    small_case(renderer, sc, scenes.default_camera(128, 96), "power-law SH1 3000 128x96", bg=(0.5, 0.5, 0.5),
               seed=5)


@pytest.mark.parametrize("dtype", [1, 2], ids=["bf16", "fp16"])
def test_backward_reduced_precision_storage(renderer, dtype):
    """Gradients with respect to the values the kernel reads (the dequantised
    attributes), in float32."""
    sc = enlarged(scenes.make_scene("C2", n=300, seed=44, sh_degree=2), by=2.0)
    small_case(renderer, sc, scenes.default_camera(64, 64), f"SH2 300 64x64 storage {dtype}", dtype=dtype, seed=6)


def test_backward_culled_gaussians_get_zero(renderer):
    """Gaussians behind the camera or off screen get exactly zero gradient."""
    sc = enlarged(scenes.make_scene("C1", n=200, seed=45, sh_degree=0))
    sc["means"][2, :5] = np.float32(-4.0)      # behind the camera
    sc["means"][0, 5:10] = np.float32(30.0)    # far off screen
    got, want = small_case(renderer, sc, scenes.default_camera(48, 48), "culled", seed=7)
    for k in GROUPS:
        assert not np.any(got[k][..., :10]), k


def test_backward_empty_frame(renderer):
    """Nothing visible: every gradient is zero."""
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C1", n=50, seed=46, sh_degree=0)
    sc["means"][2, :] = np.float32(-4.0)
    cam = scenes.default_camera(40, 24)
    dev = gs.scene_to_device(sc, 0)
    renderer.render(dev, cam, 40, 24)
    w_rgb, w_T = loss_weights(cam, 8)
    got = gpu_grads(renderer, dev, [w_rgb], [w_T])
    for k in GROUPS:
        assert not np.any(got[k]), k


def test_batched_backward_sums_views(renderer):
    """One backward over a batched render equals the oracle's gradient summed
    over the views (each view with its own size and weights)."""
    import paper_2607_15951_amd as gs
    import torch
    sc = enlarged(scenes.make_scene("C2", n=300, seed=47, sh_degree=1), by=2.0)
    cams = [scenes.default_camera(64, 48), scenes.look_at_camera([1.5, -0.4, -2.4], 50, 40),
            scenes.look_at_camera([-2.0, 0.3, -2.0], 80, 36)]
    bg = (0.1, 0.2, 0.3)
    say(f"[backward] batched: {len(cams)} views")
    dev = gs.scene_to_device(sc, 0)
    renderer.render_batched(dev, cams, background=bg)
    torch.cuda.synchronize()
    ws, wts, want = [], [], {k: 0.0 for k in GROUPS}
    for v, cam in enumerate(cams):
        o = oracle.render(sc, cam, background=bg)
        w_rgb, w_T = loss_weights(cam, 20 + v, ambiguous=oracle.ambiguous_mask(o))
        ws.append(w_rgb)
        wts.append(w_T)
        g = oracle_grads(sc, cam, w_rgb, w_T, bg, proj=o["proj"])
        for k in GROUPS:
            want[k] = want[k] + g[k]
    got = gpu_grads(renderer, dev, ws, wts)
    compare("batched 3 views", got, want)


def test_autograd_wrapper(renderer):
    """render_autograd: gradients through torch.autograd equal the oracle's,
    and a second render before the backward is refused."""
    import paper_2607_15951_amd as gs
    import torch
    sc = enlarged(scenes.make_scene("C2", n=250, seed=48, sh_degree=3), by=2.0)
    cam = scenes.default_camera(56, 40)
    o = oracle.render(sc, cam)
    w_rgb, w_T = loss_weights(cam, 9, ambiguous=oracle.ambiguous_mask(o))
    leaves = {k: torch.from_numpy(np.ascontiguousarray(sc[k], np.float32)).cuda().requires_grad_(True)
              for k in GROUPS}
    img, T = gs.render_autograd(renderer, leaves["means"], leaves["log_scales"], leaves["quats"],
                                leaves["opacity_logits"], leaves["sh"], cam, 56, 40)
    loss = (img * torch.from_numpy(w_rgb.astype(np.float32)).cuda()).sum() + \
        (T * torch.from_numpy(w_T.astype(np.float32)).cuda()).sum()
    loss.backward()
    got = {k: leaves[k].grad.cpu().numpy() for k in GROUPS}
    want = oracle_grads(sc, cam, w_rgb, w_T, (0.0, 0.0, 0.0), proj=o["proj"])
    compare("autograd SH3", got, want)
    # a stale backward is an error, not a wrong gradient
    img2, T2 = gs.render_autograd(renderer, leaves["means"], leaves["log_scales"], leaves["quats"],
                                  leaves["opacity_logits"], leaves["sh"], cam, 56, 40)
    dev = {k: v.detach() for k, v in leaves.items()}
    dev.update(sh_degree=3, attr_dtype=0)
    renderer.render(dev, cam, 56, 40)
    with pytest.raises(RuntimeError):
        img2.sum().backward()


def test_backward_rejects_bad_calls(renderer):
    import paper_2607_15951_amd as gs
    import torch
    sc = scenes.make_scene("C1", n=100, seed=49, sh_degree=0)
    cam = scenes.default_camera(32, 32)
    dev = gs.scene_to_device(sc, 0)
    w = [torch.zeros((3, 32, 32), device="cuda")]
    renderer.render(dev, cam, 32, 32, want_T=False)
    with pytest.raises(RuntimeError):
        renderer.backward(dev, w)                    # the forward kept no final_T
    renderer.render(dev, cam, 32, 32)
    other = gs.scene_to_device(sc, 0)
    with pytest.raises(RuntimeError):
        renderer.backward(other, w)                  # not the scene of the last render
    renderer.backward(dev, w)
    torch.cuda.synchronize()


def test_backward_c3_full_size_sampled_tiles(renderer):
    """The bench workload (3M Gaussians, SH3, 1920x1080) with the loss on a
    sample of tiles: the Gaussians listed in those tiles get the oracle's
    gradient, every other Gaussian exactly zero."""
    import paper_2607_15951_amd as gs
    import torch
    scene = scenes.make_scene("C3")
    cam = scenes.make_cameras("C3")[0]
    W, H = cam["width"], cam["height"]
    tx = (W + TILE - 1) // TILE
    say(f"[backward] C3 full size: render")
    dev = gs.scene_to_device(scene, 0)
    renderer.render(dev, cam, W, H)
    torch.cuda.synchronize()
    projg = renderer.projection()
    g_rect = projg["rect"].cpu().numpy().view(np.uint16).astype(np.int32)
    g = dict(splats=projg["splats"].cpu().numpy(),
             depth_key=projg["depth_key"].cpu().numpy().view(np.uint32),
             radius=projg["radius"].cpu().numpy(),
             tiles_touched=projg["tiles_touched"].cpu().numpy().view(np.uint32), rect=g_rect)
    say(f"[backward] C3 full size: oracle projection")
    p = oracle.project(scene, cam)
    amb = check_projection(g, p, "C3 backward")
    differ = [int(i) for i in amb if not np.array_equal(g_rect[i], p["rect"][:, i])]
    counts = oracle.tile_counts(p).astype(np.int64)
    rng = np.random.default_rng(77)
    cand = [0, tx - 1, (H // TILE // 2) * tx + tx // 2] + [int(t) for t in np.argsort(-counts)[:1]] + \
        [int(t) for t in rng.integers(0, len(counts), 4)]
    bad = set()
    for i in differ:
        for r in (g_rect[i], p["rect"][:, i]):
            for yy in range(r[1], r[3]):
                bad.update(range(yy * tx + r[0], yy * tx + r[2]))
    tiles = sorted({t for t in cand if t not in bad})
    # pixel ambiguity of the sampled tiles, from the oracle composite
    amb_px = np.zeros((H, W), bool)
    members = set()
    for t in tiles:
        lst = oracle.tile_list(p, t)
        members.update(int(i) for i in lst)
        x0, y0 = (t % tx) * TILE, (t // tx) * TILE
        ys, xs = np.mgrid[y0:min(y0 + TILE, H), x0:min(x0 + TILE, W)]
        _, marg = oracle.composite_pixels(p, xs.ravel(), ys.ravel(), lst)
        amb_px[ys.ravel(), xs.ravel()] = (marg[:, 0] < oracle.ALPHA_MARGIN) | (marg[:, 1] < oracle.T_MARGIN)
    w_rgb, w_T = loss_weights(cam, 10, ambiguous=amb_px, tiles=tiles)
    say(f"[backward] C3 full size: GPU backward, tiles {tiles}, {len(members)} Gaussians listed")
    got = gpu_grads(renderer, dev, [w_rgb], [w_T])
    del dev
    U = np.array(sorted(members), np.int64)
    sub = {k: np.ascontiguousarray(scene[k][..., U]) for k in GROUPS}
    sub["sh_degree"] = scene["sh_degree"]
    psub = oracle.project(sub, cam)
    want = oracle_grads(sub, cam, w_rgb, w_T, (0.0, 0.0, 0.0), proj=psub, tiles=tiles)
    compare(f"C3 full size, {len(tiles)} tiles", got, want, idx=U)
    outside = np.ones(scene["means"].shape[1], bool)
    outside[U] = False
    for k in GROUPS:
        assert not np.any(got[k][..., outside]), f"{k}: gradient on a Gaussian listed in no sampled tile"


def test_graph_backward_follows_the_launched_views(renderer):
    """A backward after gs_graph_launch differentiates the cameras and outputs
    of that launch (after gs_graph_set_views too), equal to the oracle's
    gradient summed over those views; it leaves the graph's own view table
    alone, so the next launch still renders the new cameras (against the
    oracle as well)."""
    import paper_2607_15951_amd as gs
    import torch
    from parity import check_image
    sc = enlarged(scenes.make_scene("C2", n=300, seed=50, sh_degree=1), by=2.0)
    cams1 = [scenes.default_camera(64, 48), scenes.look_at_camera([1.5, -0.4, -2.4], 50, 40)]
    cams2 = [scenes.look_at_camera([-1.2, 0.5, -2.6], 64, 48), scenes.look_at_camera([0.4, 1.6, -2.3], 50, 40)]
    dev = gs.scene_to_device(sc, 0)
    r = gs.Renderer(0)
    try:
        gr = r.graph(dev, cams1, pair_capacity=200_000)
        gr.set_views(cams2)
        outs = gr.launch()
        torch.cuda.synchronize()
        ws, wts, want = [], [], {k: 0.0 for k in GROUPS}
        for v, cam in enumerate(cams2):
            o = oracle.render(sc, cam)
            check_image({"image": outs[v]["image"].cpu().numpy().astype(np.float64),
                         "final_T": outs[v]["final_T"].cpu().numpy().astype(np.float64),
                         "n_contrib": outs[v]["n_contrib"].cpu().numpy()}, o, f"graph view {v}")
            w_rgb, w_T = loss_weights(cam, 30 + v, ambiguous=oracle.ambiguous_mask(o))
            ws.append(w_rgb)
            wts.append(w_T)
            g = oracle_grads(sc, cam, w_rgb, w_T, (0.0, 0.0, 0.0), proj=o["proj"])
            for k in GROUPS:
                want[k] = want[k] + g[k]
        got = gpu_grads(r, dev, ws, wts)
        compare("graph launch, new views", got, want)
        first = [o["image"].clone() for o in outs]
        for o in outs:
            o["image"].fill_(-1.0)
        gr.launch()
        torch.cuda.synchronize()
        for o, f in zip(outs, first):
            assert torch.equal(o["image"], f), "the launch after a backward rendered other views"
        gr.close()
    finally:
        r.close()


def test_autograd_refuses_outputs_modified_in_place(renderer):
    """The image and final T that the backward reads are saved for backward:
    editing either in place makes autograd raise instead of returning wrong
    gradients."""
    import paper_2607_15951_amd as gs
    import torch
    sc = enlarged(scenes.make_scene("C1", n=120, seed=51, sh_degree=0))
    cam = scenes.default_camera(40, 32)
    leaves = {k: torch.from_numpy(np.ascontiguousarray(sc[k], np.float32)).cuda().requires_grad_(True)
              for k in GROUPS}
    img, T = gs.render_autograd(renderer, leaves["means"], leaves["log_scales"], leaves["quats"],
                                leaves["opacity_logits"], leaves["sh"], cam, 40, 32)
    img.clamp_(0.0, 0.5)
    with pytest.raises(RuntimeError, match="inplace"):
        img.sum().backward()
