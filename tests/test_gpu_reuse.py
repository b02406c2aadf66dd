"""Reuse of the previous frame's depth order (GS_RENDER_REUSE_ORDER).

The flag changes the work, never the result: along orbits of several step
sizes, after a teleport, and when a few Gaussians move, every frame rendered
with it must equal the same frame rendered without it, bit for bit (image,
final T, n_contrib, tile offsets and values) -- and the plain render is the
one the oracle parity tests check.  The reported outcome must match what the
order allows: a static camera reuses with no descent, a few nudged Gaussians
are repaired locally, a Gaussian thrown far in depth or a teleport falls back
to the radix sort.
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
    lists = renderer.lists(keys=False)
    return {"offsets": lists["tile_offsets"].cpu().numpy().copy(), "values": lists["values"].cpu().numpy().copy(),
            "image": out["image"].cpu().numpy().view(np.uint32).copy(),
            "T": out["final_T"].cpu().numpy().view(np.uint32).copy(), "nc": out["n_contrib"].cpu().numpy().copy()}


def check_orbit(renderer, dev, angles, W, H, label):
    outcomes = []
    for k, a in enumerate(angles):
        cam = scenes.orbit_camera(a, W, H)
        out = renderer.render(dev, cam, W, H, reuse_order=True)
        got = snapshot(renderer, out)
        rep = renderer.order_reuse() if k > 0 else None
        want = snapshot(renderer, renderer.render(dev, cam, W, H))
        for key in want:
            assert np.array_equal(got[key], want[key]), f"{label} frame {k} ({a} deg): {key} differs"
        outcomes.append(rep)
    say(f"[reuse] {label}: " + ", ".join(f"{o['reused']:d}/{o['descents']}" for o in outcomes[1:]))
    return outcomes[1:]


def test_orbit_steps_and_teleport(renderer):
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C3", n=200_000, seed=51)
    dev = gs.scene_to_device(sc)
    W, H = 480, 270
    static = check_orbit(renderer, dev, [0.0, 0.0, 0.0], W, H, "static")
    assert all(o["reused"] and o["descents"] == 0 for o in static)
    check_orbit(renderer, dev, [0.0, 0.001, 0.002], W, H, "orbit 0.001 deg")
    check_orbit(renderer, dev, [0.0, 0.01, 0.02, 0.03], W, H, "orbit 0.01 deg")
    check_orbit(renderer, dev, [0.0, 0.5, 1.0], W, H, "orbit 0.5 deg")
    tele = check_orbit(renderer, dev, [0.0, 137.0, 271.0], W, H, "teleport")
    assert not any(o["reused"] for o in tele)


def test_nudged_gaussians_are_repaired_locally(renderer):
    """A static camera while a few Gaussians move a little in depth (a few
    descents: the local repair) or one moves far (the repair fails its check:
    the radix sort)."""
    import paper_2607_15951_amd as gs
    import torch
    sc = scenes.make_scene("C3", n=200_000, seed=57)
    dev = gs.scene_to_device(sc)
    W, H = 480, 270
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    rng = np.random.default_rng(8)
    for label, count, dz in (("nudge", 200, 2e-4), ("throw", 1, 1.5)):
        idx = torch.from_numpy(rng.choice(200_000, count, replace=False)).cuda()
        dev["means"][2, idx] += dz
        got = snapshot(renderer, renderer.render(dev, cam, W, H, reuse_order=True))
        rep = renderer.order_reuse()
        want = snapshot(renderer, renderer.render(dev, cam, W, H))
        say(f"[reuse] {label}: {rep}")
        for key in want:
            assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"
        assert 0 < rep["descents"] <= 200_000 // 256, rep
        assert rep["reused"] == (label == "nudge"), rep


def test_reuse_is_ignored_when_it_cannot_apply(renderer):
    """A different Gaussian count, a batched render in between, or no render
    before: the flag is accepted, the sort runs from scratch."""
    import paper_2607_15951_amd as gs
    W, H = 160, 96
    cam = scenes.default_camera(W, H)
    a = gs.scene_to_device(scenes.make_scene("C2", n=20_000, seed=52))
    b = gs.scene_to_device(scenes.make_scene("C2", n=25_000, seed=53))
    fresh = gs.Renderer(0)
    try:
        fresh.render(a, cam, W, H, reuse_order=True)   # first render of the context
        with pytest.raises(RuntimeError):
            fresh.order_reuse()
    finally:
        fresh.close()
    renderer.render(a, cam, W, H)
    renderer.render(b, cam, W, H, reuse_order=True)    # other n
    with pytest.raises(RuntimeError):
        renderer.order_reuse()
    renderer.render_batched(b, [cam, scenes.orbit_camera(5.0, W, H)])
    out = renderer.render(b, cam, W, H, reuse_order=True)   # after a batched render
    with pytest.raises(RuntimeError):
        renderer.order_reuse()
    got = snapshot(renderer, out)
    want = snapshot(renderer, renderer.render(b, cam, W, H))
    for key in want:
        assert np.array_equal(got[key], want[key]), key


def test_other_scene_of_same_size(renderer):
    """Same count, different Gaussians: the old order is only a starting
    point, the result is still this scene's order."""
    import paper_2607_15951_amd as gs
    W, H = 200, 120
    cam = scenes.default_camera(W, H)
    a = gs.scene_to_device(scenes.make_scene("C2", n=30_000, seed=54))
    b = gs.scene_to_device(scenes.make_scene("C3", n=30_000, seed=55))
    renderer.render(a, cam, W, H)
    got = snapshot(renderer, renderer.render(b, cam, W, H, reuse_order=True))
    assert not renderer.order_reuse()["reused"]
    want = snapshot(renderer, renderer.render(b, cam, W, H))
    for key in want:
        assert np.array_equal(got[key], want[key]), key


def test_graph_with_reuse_follows_camera_changes(renderer):
    """A captured render with the flag: replays along an orbit match eager
    renders of the same cameras."""
    import paper_2607_15951_amd as gs
    import torch
    W, H = 256, 144
    sc = scenes.make_scene("C3", n=80_000, seed=56)
    dev = gs.scene_to_device(sc)
    cams = [scenes.orbit_camera(a, W, H) for a in (0.0, 0.02, 0.04, 3.0)]
    renderer.render(dev, cams[0], W, H)
    cap = int(renderer.list_info()["num_pairs"] * 1.5) + 4096
    gr = renderer.graph(dev, [cams[0]], pair_capacity=cap, reuse_order=True)
    try:
        for c in cams:
            gr.set_views([c])
            gr.launch()
            torch.cuda.synchronize()
            img = gr.outs[0]["image"].cpu().numpy().copy()
            ref = gs.Renderer(0)
            try:
                want = ref.render(dev, c, W, H)["image"].cpu().numpy()
            finally:
                ref.close()
            assert np.array_equal(img.view(np.uint32), want.view(np.uint32))
    finally:
        gr.close()


def _result(renderer, out):
    """gpu_render-style result dict of the renderer's last render."""
    import torch
    torch.cuda.synchronize()
    lists = renderer.lists(keys=True)
    proj = renderer.projection()
    torch.cuda.synchronize()
    return dict(image=out["image"].cpu().numpy().astype(np.float64),
                final_T=out["final_T"].cpu().numpy().astype(np.float64), n_contrib=out["n_contrib"].cpu().numpy(),
                values=lists["values"].cpu().numpy().view(np.uint32),
                tile_offsets=lists["tile_offsets"].cpu().numpy().view(np.uint32),
                keys=lists["keys"].cpu().numpy().view(np.uint64), num_pairs=lists["num_pairs"],
                splats=proj["splats"].cpu().numpy(), depth_key=proj["depth_key"].cpu().numpy().view(np.uint32),
                radius=proj["radius"].cpu().numpy(), tiles_touched=proj["tiles_touched"].cpu().numpy().view(np.uint32),
                rect=proj["rect"].cpu().numpy().view(np.uint16).astype(np.int32))


def test_reused_frames_match_the_oracle(renderer):
    """Frames whose depth sort was skipped (static camera: the previous order
    reused as is; a few nudged Gaussians: the order repaired in place) against
    the oracle directly: projection, whole lists, image."""
    import paper_2607_15951_amd as gs
    import torch
    from parity import oracle_view_parity
    sc = scenes.make_scene("C3", n=60_000, seed=58)
    dev = gs.scene_to_device(sc)
    W, H = 320, 180
    cam = scenes.default_camera(W, H)
    renderer.render(dev, cam, W, H)
    out = renderer.render(dev, cam, W, H, reuse_order=True)
    g = _result(renderer, out)
    assert renderer.order_reuse() == {"reused": True, "descents": 0}
    say(f"[reuse] static frame vs oracle: {oracle_view_parity(g, sc, cam, 'reused order')}")
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(60_000, 60, replace=False))
    sc2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    sc2["means"][2, idx] += np.float32(2e-4)
    dev["means"].copy_(torch.from_numpy(sc2["means"]).cuda())
    out = renderer.render(dev, cam, W, H, reuse_order=True)
    g = _result(renderer, out)
    rep = renderer.order_reuse()
    assert rep["reused"] and rep["descents"] > 0, rep
    say(f"[reuse] repaired frame ({rep}) vs oracle: {oracle_view_parity(g, sc2, cam, 'repaired order')}")
