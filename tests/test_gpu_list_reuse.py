"""Reuse of the previous frame's tile lists (GS_RENDER_REUSE_LISTS).

The lists depend only on the depth keys, the tile rectangles and the image
size, so when the projection finds every key and rectangle unchanged the
previous lists are this frame's.  The flag changes the work, never the
result: a static camera, colour and SH edits, and a moving camera must all
give, bit for bit, what the same render gives without the flag (image, final
T, n_contrib, tile offsets, values and keys), and a frame drawn from kept
lists is checked against the oracle directly.  The reported outcome must
match what changed; the flag is ignored where it cannot apply.
"""
import sys

import numpy as np
import pytest

import scenes


pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


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


def snapshot(renderer, out):
    import torch
    torch.cuda.synchronize()
    lists = renderer.lists(keys=True)
    return {"offsets": lists["tile_offsets"].cpu().numpy().copy(), "values": lists["values"].cpu().numpy().copy(),
            "keys": lists["keys"].cpu().numpy().copy(),
            "image": out["image"].cpu().numpy().view(np.uint32).copy(),
            "T": out["final_T"].cpu().numpy().view(np.uint32).copy(), "nc": out["n_contrib"].cpu().numpy().copy()}


def plain(dev, cam, W, H):
    """The same frame from a fresh context, without any flag."""
    import paper_2607_15951_amd as gs
    r = gs.Renderer(0)
    try:
        return snapshot(r, r.render(dev, cam, W, H))
    finally:
        r.close()


def same(got, want, label):
    for key in want:
        assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"


def test_static_camera_and_colour_edits_keep_the_lists(renderer):
    import paper_2607_15951_amd as gs
    import torch
    W, H = 320, 180
    sc = scenes.make_scene("C3", n=60_000, seed=71)
    dev = gs.scene_to_device(sc)
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True))
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
    same(got, plain(dev, cam, W, H), "static camera")
    # colour and SH edits leave keys and rectangles alone
    rng = np.random.default_rng(3)
    dev["sh"].mul_(0.5).add_(torch.from_numpy(rng.normal(0.0, 0.1, size=tuple(dev["sh"].shape))
                                              .astype(np.float32)).cuda())
    got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True))
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
    same(got, plain(dev, cam, W, H), "SH edit")
    # an opacity edit changes neither keys nor rectangles either (the radius
    # is the covariance's 3 sigma); whatever the outcome, the result holds
    dev["opacity_logits"].sub_(0.7)
    got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True))
    rep = renderer.list_reuse()
    say(f"[lists] opacity edit: {rep}")
    same(got, plain(dev, cam, W, H), "opacity edit")
    # three kept frames in a row stay kept
    for k in range(3):
        renderer.render(dev, cam, W, H, reuse_lists=True)
        assert renderer.list_reuse()["reused"], k


@pytest.mark.parametrize("dtype_name", ["GS_BF16", "GS_F16"])
def test_kept_lists_with_reduced_storage(renderer, dtype_name):
    """BF16 and FP16 attribute storage: an SH edit keeps the lists, and the
    frame is the plain render's."""
    import paper_2607_15951_amd as gs
    W, H = 224, 160
    sc = scenes.make_scene("C3", n=30_000, seed=77)
    dev = gs.scene_to_device(sc, getattr(gs, dtype_name))
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    dev["sh"].mul_(-0.75)
    got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True))
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
    same(got, plain(dev, cam, W, H), f"{dtype_name} SH edit")


def test_moving_geometry_rebuilds_the_lists(renderer):
    """A camera step, or a few moved Gaussians: the comparison counts them,
    the lists are rebuilt, and the frame is the plain render's."""
    import paper_2607_15951_amd as gs
    import torch
    W, H = 256, 144
    sc = scenes.make_scene("C3", n=50_000, seed=72)
    dev = gs.scene_to_device(sc)
    outcomes = []
    for k, a in enumerate((0.0, 0.01, 0.01, 0.5)):
        cam = scenes.orbit_camera(a, W, H)
        got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True, reuse_order=True))
        if k > 0:
            outcomes.append(renderer.list_reuse())
        same(got, plain(dev, cam, W, H), f"orbit {a} deg")
    say(f"[lists] orbit: {outcomes}")
    assert outcomes[0]["changed"] > 0 and not outcomes[0]["reused"]
    assert outcomes[1] == {"reused": True, "changed": 0}   # the same camera again
    assert outcomes[2]["changed"] > outcomes[0]["changed"] // 2 and not outcomes[2]["reused"]
    # a handful of Gaussians moved in depth: exactly those are counted
    cam = scenes.orbit_camera(0.5, W, H)
    proj = renderer.projection()
    keys0 = proj["depth_key"].cpu().numpy().view(np.uint32).copy()
    rect0 = proj["rect"].cpu().numpy().copy()
    idx = np.array([5, 1234, 40_000])
    means = sc["means"].copy()
    means[2, idx] += np.float32(0.05)
    dev["means"].copy_(torch.from_numpy(means).cuda())
    got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_lists=True))
    proj = renderer.projection()
    keys1 = proj["depth_key"].cpu().numpy().view(np.uint32)
    rect1 = proj["rect"].cpu().numpy()
    moved = int(np.count_nonzero((keys0 != keys1) | np.any(rect0 != rect1, axis=-1)))
    rep = renderer.list_reuse()
    say(f"[lists] three moved Gaussians: {rep}, by the outputs {moved}")
    assert rep == {"reused": False, "changed": moved} and 1 <= moved <= 3
    same(got, plain(dev, cam, W, H), "moved Gaussians")


def test_kept_lists_match_the_oracle(renderer):
    """A frame drawn from kept lists after an SH edit, against the oracle
    directly: projection, whole lists, image."""
    import paper_2607_15951_amd as gs
    import torch
    from parity import oracle_view_parity
    W, H = 320, 180
    sc = scenes.make_scene("C3", n=60_000, seed=73)
    dev = gs.scene_to_device(sc)
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    sc2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    sc2["sh"] = (sc["sh"] * np.float32(-0.8)).astype(np.float32)
    dev["sh"].copy_(torch.from_numpy(sc2["sh"]).cuda())
    out = renderer.render(dev, cam, W, H, reuse_lists=True)
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
    torch.cuda.synchronize()
    lists = renderer.lists(keys=True)
    proj = renderer.projection()
    torch.cuda.synchronize()
    g = dict(image=out["image"].cpu().numpy().astype(np.float64),
             final_T=out["final_T"].cpu().numpy().astype(np.float64), n_contrib=out["n_contrib"].cpu().numpy(),
             values=lists["values"].cpu().numpy().view(np.uint32),
             tile_offsets=lists["tile_offsets"].cpu().numpy().view(np.uint32),
             keys=lists["keys"].cpu().numpy().view(np.uint64), num_pairs=lists["num_pairs"],
             splats=proj["splats"].cpu().numpy(), depth_key=proj["depth_key"].cpu().numpy().view(np.uint32),
             radius=proj["radius"].cpu().numpy(), tiles_touched=proj["tiles_touched"].cpu().numpy().view(np.uint32),
             rect=proj["rect"].cpu().numpy().view(np.uint16).astype(np.int32))
    say(f"[lists] kept lists after an SH edit vs oracle: {oracle_view_parity(g, sc2, cam, 'kept lists')}")


def test_backward_after_kept_lists(renderer):
    """The backward of a frame drawn from kept lists equals the backward of
    the plain frame (float atomics: to rounding)."""
    import paper_2607_15951_amd as gs
    import torch
    W, H = 192, 128
    sc = scenes.make_scene("C3", n=20_000, seed=74)
    dev = gs.scene_to_device(sc)
    cam = scenes.default_camera(W, H)
    gimg = torch.from_numpy(np.random.default_rng(5).normal(size=(3, H, W)).astype(np.float32)).cuda()
    renderer.render(dev, cam, W, H)
    want = {k: v.cpu().numpy() for k, v in renderer.backward(dev, [gimg]).items()}
    renderer.render(dev, cam, W, H, reuse_lists=True)
    assert renderer.list_reuse()["reused"]
    got = {k: v.cpu().numpy() for k, v in renderer.backward(dev, [gimg]).items()}
    for k in want:
        err = np.linalg.norm(got[k] - want[k]) / max(np.linalg.norm(want[k]), 1e-30)
        assert err < 1e-5, (k, err)


def test_graph_replays_keep_the_lists(renderer):
    """A captured render with the flag: replays of a static camera keep the
    lists (the decision is taken on the device), a camera change rebuilds
    them, and every replay matches the eager render of its camera."""
    import paper_2607_15951_amd as gs
    import torch
    W, H = 256, 144
    sc = scenes.make_scene("C3", n=60_000, seed=78)
    dev = gs.scene_to_device(sc)
    cams = [scenes.orbit_camera(a, W, H) for a in (0.0, 0.0, 0.2, 0.2, 0.2)]
    renderer.render(dev, cams[0], W, H)
    cap = int(renderer.list_info()["num_pairs"] * 1.5) + 4096
    gr = renderer.graph(dev, [cams[0]], pair_capacity=cap, reuse_lists=True)
    outcomes = []
    try:
        for k, c in enumerate(cams):
            gr.set_views([c])
            if k == 3:
                dev["sh"].mul_(0.5)   # a colour edit between two replays of one camera
            gr.launch()
            torch.cuda.synchronize()
            outcomes.append(renderer.list_reuse())
            img = gr.outs[0]["image"].cpu().numpy().view(np.uint32).copy()
            want = plain(dev, c, W, H)["image"]
            assert np.array_equal(img, want), f"replay {k}"
    finally:
        gr.close()
    say(f"[lists] graph replays: {outcomes}")
    assert [o["reused"] for o in outcomes] == [True, True, False, True, True], outcomes


def test_batched_views_keep_the_lists(renderer):
    """A batched render of three views of different sizes: unchanged views
    keep all lists, one moved camera rebuilds them, and every view matches its
    plain single render."""
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C3", n=40_000, seed=80)
    dev = gs.scene_to_device(sc)
    sizes = [(160, 96), (256, 144), (96, 200)]
    cams = [scenes.orbit_camera(20.0 * k, w, h) for k, (w, h) in enumerate(sizes)]
    renderer.render_batched(dev, cams)
    outcomes = []
    for step, moved in ((0, False), (1, True), (2, False)):
        if moved:
            w, h = sizes[1]
            cams[1] = scenes.orbit_camera(20.5, w, h)
        dev["sh"].mul_(0.9)
        outs = renderer.render_batched(dev, cams, reuse_lists=True)
        outcomes.append(renderer.list_reuse())
        for k, (c, o) in enumerate(zip(cams, outs)):
            w, h = sizes[k]
            want = plain(dev, c, w, h)
            got = o["image"].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, want["image"]), f"step {step} view {k}: image"
            assert np.array_equal(o["n_contrib"].cpu().numpy(), want["nc"]), f"step {step} view {k}: n_contrib"
    say(f"[lists] batched: {outcomes}")
    assert outcomes[0] == {"reused": True, "changed": 0}
    assert not outcomes[1]["reused"] and outcomes[1]["changed"] > 0
    assert outcomes[2] == {"reused": True, "changed": 0}


def test_capacity_renders_keep_the_lists(renderer):
    """Renders with one pair capacity compare with each other; the frame of
    kept lists matches the plain capacity render."""
    import paper_2607_15951_amd as gs
    W, H = 200, 120
    sc = scenes.make_scene("C3", n=30_000, seed=79)
    dev = gs.scene_to_device(sc)
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    cap = int(renderer.list_info()["num_pairs"] * 1.2) + 1024
    renderer.render(dev, cam, W, H, pair_capacity=cap)
    got = snapshot(renderer, renderer.render(dev, cam, W, H, pair_capacity=cap, reuse_lists=True))
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
    same(got, plain(dev, cam, W, H), "capacity render")


def test_list_reuse_is_ignored_when_it_cannot_apply(renderer):
    """First render of a context, another image size, Gaussian count, pair
    capacity or view count in between: no comparison is made, and the result
    is unchanged."""
    import paper_2607_15951_amd as gs
    W, H = 160, 96
    cam = scenes.default_camera(W, H)
    a = gs.scene_to_device(scenes.make_scene("C2", n=20_000, seed=75))
    b = gs.scene_to_device(scenes.make_scene("C2", n=25_000, seed=76))
    fresh = gs.Renderer(0)
    try:
        fresh.render(a, cam, W, H, reuse_lists=True)   # first render of the context
        with pytest.raises(RuntimeError):
            fresh.list_reuse()
    finally:
        fresh.close()

    def not_compared(out, dev, c, w, h, label):
        with pytest.raises(RuntimeError):
            renderer.list_reuse()
        same(snapshot(renderer, out), plain(dev, c, w, h), label)

    renderer.render(a, cam, W, H)
    not_compared(renderer.render(b, cam, W, H, reuse_lists=True), b, cam, W, H, "other n")
    cam2 = scenes.default_camera(W + 16, H)
    not_compared(renderer.render(b, cam2, W + 16, H, reuse_lists=True), b, cam2, W + 16, H, "other size")
    renderer.render_batched(b, [cam, scenes.orbit_camera(5.0, W, H)])
    not_compared(renderer.render(b, cam, W, H, reuse_lists=True), b, cam, W, H, "after a batched render")
    cap = int(renderer.list_info()["num_pairs"] * 2) + 4096
    renderer.render(b, cam, W, H, pair_capacity=cap)
    not_compared(renderer.render(b, cam, W, H, reuse_lists=True), b, cam, W, H, "capacity lists, then eager")
    renderer.render(b, cam, W, H)
    not_compared(renderer.render(b, cam, W, H, reuse_lists=True, pair_capacity=cap), b, cam, W, H,
                 "eager lists, then a pair capacity")
    # and once the conditions hold again, the lists are kept
    renderer.render(b, cam, W, H)
    renderer.render(b, cam, W, H, reuse_lists=True)
    assert renderer.list_reuse() == {"reused": True, "changed": 0}
