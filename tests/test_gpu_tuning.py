"""Launch-shape tuning (gs_set_tuning, gs_autotune) on the GPU.

Every supported shape must give the same render bit for bit (image, final T,
n_contrib, tile offsets and values), eager and with a pair capacity, single
and batched; the default shape is the one the oracle parity tests check.
The autotuner must return one of its candidates and leave the results
unchanged.
"""
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

CANDIDATES = {"sort_items": (4, 8, 16), "bin_row_items": (4, 8, 16), "bin_tile_items": (8, 16, 32),
              "blend_tile_group": (-1, 0, 1, 2, 4, 8, 16, 32, 64), "blend_batch": (128, 256, 512)}
DEFAULT = {"sort_items": 8, "bin_row_items": 8, "bin_tile_items": 16, "blend_tile_group": 0, "blend_batch": 256}


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


def snapshot(renderer, outs):
    import torch
    torch.cuda.synchronize()
    lists = renderer.lists(keys=False)
    res = {"offsets": lists["tile_offsets"].cpu().numpy().copy(), "values": lists["values"].cpu().numpy().copy()}
    for v, o in enumerate(outs):
        res[f"image{v}"] = o["image"].cpu().numpy().view(np.uint32).copy()
        res[f"T{v}"] = o["final_T"].cpu().numpy().view(np.uint32).copy()
        res[f"nc{v}"] = o["n_contrib"].cpu().numpy().copy()
    return res


def render_all(renderer, dev, cams, capacity):
    if len(cams) == 1:
        c = cams[0]
        return [renderer.render(dev, c, c["width"], c["height"], pair_capacity=capacity)]
    return renderer.render_batched(dev, cams, pair_capacity=capacity)


def shapes():
    out = []
    for k, vals in CANDIDATES.items():
        for v in vals:
            if v != DEFAULT[k]:
                out.append({k: v})
    out.append({k: vals[0] for k, vals in CANDIDATES.items()})
    out.append({k: vals[-1] for k, vals in CANDIDATES.items()})
    return out


CASES = {
    "C2-dist 40k 333x197": lambda: (scenes.make_scene("C2", n=40_000, seed=21), [scenes.default_camera(333, 197)]),
    "C3-dist 60k rotated 400x240": lambda: (scenes.make_scene("C3", n=60_000, seed=31),
                                            [scenes.look_at_camera([1.2, -0.8, -2.7], 400, 240)]),
    "batched 3 views": lambda: (scenes.make_scene("C2", n=30_000, seed=23),
                                [scenes.default_camera(200, 120), scenes.look_at_camera([1.5, -0.4, -2.4], 96, 64),
                                 scenes.look_at_camera([-2.0, 0.3, -2.0], 300, 180)]),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("capacity", [0, 1], ids=["eager", "capacity"])
def test_every_shape_gives_identical_results(renderer, case, capacity):
    import paper_2607_15951_amd as gs
    sc, cams = CASES[case]()
    dev = gs.scene_to_device(sc)
    renderer.set_tuning(**DEFAULT)
    cap = 0
    if capacity:
        render_all(renderer, dev, cams, 0)
        cap = int(renderer.list_info()["num_pairs"] * 1.3) + 1024
    outs = render_all(renderer, dev, cams, cap)
    want = snapshot(renderer, outs)
    say(f"[tuning] {case} capacity={cap}: {len(want['values'])} pairs, {len(shapes())} shapes")
    try:
        for sh in shapes():
            renderer.set_tuning(**DEFAULT)
            renderer.set_tuning(**sh)
            got = snapshot(renderer, render_all(renderer, dev, cams, cap))
            for k in want:
                assert np.array_equal(got[k], want[k]), f"{case}: {k} differs with {sh}"
    finally:
        renderer.set_tuning(**DEFAULT)


def test_set_tuning_rejects_unsupported_values(renderer):
    renderer.set_tuning(**DEFAULT)
    for bad in ({"sort_items": 5}, {"bin_row_items": 32}, {"bin_tile_items": 4}, {"blend_tile_group": -2},
                {"blend_tile_group": 65}, {"blend_batch": 192}):
        with pytest.raises(RuntimeError):
            renderer.set_tuning(**bad)
        assert renderer.tuning() == DEFAULT


def test_autotune_returns_a_candidate_and_keeps_results(renderer):
    import paper_2607_15951_amd as gs
    sc, cams = CASES["batched 3 views"]()
    dev = gs.scene_to_device(sc)
    renderer.set_tuning(**DEFAULT)
    want = snapshot(renderer, render_all(renderer, dev, cams, 0))
    try:
        res = renderer.autotune(dev, cams, reps=2)
        say(f"[tuning] autotune: {res['tuning']}")
        for k, v in res["tuning"].items():
            assert v in CANDIDATES[k], (k, v)
        assert renderer.tuning() == res["tuning"]
        assert len(res["candidates_ms"]) == len(gs.TUNE_CANDIDATES)
        assert all(ms > 0 for _, _, ms in res["candidates_ms"])
        got = snapshot(renderer, render_all(renderer, dev, cams, 0))
        for k in want:
            assert np.array_equal(got[k], want[k]), f"{k} differs after autotune"
    finally:
        renderer.set_tuning(**DEFAULT)


def test_backward_with_other_tile_groups(renderer):
    """The backward deals tiles like its render; gradients agree to float
    atomics' reordering."""
    import paper_2607_15951_amd as gs
    import torch
    sc = scenes.make_scene("C2", n=5_000, seed=24, sh_degree=1)
    cam = scenes.default_camera(160, 96)
    dev = gs.scene_to_device(sc)
    rng = np.random.default_rng(3)
    gi = torch.from_numpy(rng.uniform(-1, 1, (3, 96, 160)).astype(np.float32)).cuda()
    ref = None
    try:
        for group in (0, 16, 1, 64, -1):
            renderer.set_tuning(blend_tile_group=group)
            renderer.render(dev, cam, 160, 96)
            g = {k: v.cpu().numpy() for k, v in renderer.backward(dev, [gi]).items()}
            if ref is None:
                ref = g
                continue
            for k in g:
                scale = float(np.abs(ref[k]).max()) or 1.0
                assert float(np.abs(g[k] - ref[k]).max()) <= 1e-5 * scale, (group, k)
    finally:
        renderer.set_tuning(**DEFAULT)


def test_heaviest_first_order_from_length_then_history(renderer):
    """blend_tile_group 0 on a fresh context: the first render orders its
    tiles by list length, the next ones by the previous render's per-tile
    work, and a render of another size falls back to list length; every one
    equals the default dispatch bit for bit."""
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=40_000, seed=25)
    dev = gs.scene_to_device(sc)
    big, small = scenes.default_camera(333, 197), scenes.default_camera(128, 72)
    renderer.set_tuning(**DEFAULT)
    want_big = snapshot(renderer, render_all(renderer, dev, [big], 0))
    want_small = snapshot(renderer, render_all(renderer, dev, [small], 0))
    fresh = gs.Renderer(0)
    try:
        fresh.set_tuning(blend_tile_group=0)
        for cam, want in ((big, want_big), (big, want_big), (small, want_small), (big, want_big)):
            got = snapshot(fresh, render_all(fresh, dev, [cam], 0))
            for k in want:
                assert np.array_equal(got[k], want[k]), f"{cam['width']}x{cam['height']}: {k} differs"
    finally:
        fresh.close()


def test_persistent_queue_in_graph_replays_and_noalloc(renderer):
    """blend_tile_group -1 (a persistent grid draining the heaviest-first
    queue, whose head the frame's set-up launch clears): graph replays, with
    eager work between them, and the no-allocation render each equal the
    default dispatch bit for bit."""
    import torch
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=30_000, seed=26)
    dev = gs.scene_to_device(sc)
    cams = [scenes.default_camera(200, 120), scenes.look_at_camera([1.5, -0.4, -2.4], 96, 64),
            scenes.look_at_camera([-2.0, 0.3, -2.0], 300, 180)]
    renderer.set_tuning(**DEFAULT)
    want = [{k: v.clone() for k, v in o.items()} for o in renderer.render_batched(dev, cams)]
    cap = int(renderer.list_info()["num_pairs"] * 1.3) + 1024
    c0 = cams[0]
    want0 = {k: v.clone() for k, v in renderer.render(dev, c0, c0["width"], c0["height"]).items()}
    r = gs.Renderer(0)
    try:
        r.set_tuning(blend_tile_group=-1)
        gr = r.graph(dev, cams, pair_capacity=cap)
        for rep in range(3):
            for o in gr.outs:
                o["image"].fill_(-1.0)
            torch.cuda.synchronize()
            gr.launch()
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()   # eager work between replays
            for v, (o, w) in enumerate(zip(gr.outs, want)):
                for k in ("image", "final_T", "n_contrib"):
                    assert torch.equal(o[k], w[k]), f"replay {rep} view {v} {k}"
        gr.close()
        say("[tuning] queue blend: 3 graph replays equal the default dispatch")
        out = {"image": torch.full((3, c0["height"], c0["width"]), -2.0, device="cuda"),
               "final_T": torch.full((c0["height"], c0["width"]), -2.0, device="cuda"),
               "n_contrib": torch.full((c0["height"], c0["width"]), -2, dtype=torch.int32, device="cuda")}
        for _ in range(2):
            r.render_noalloc(dev, c0, c0["width"], c0["height"], out)
            torch.cuda.synchronize()
            for k in ("image", "final_T", "n_contrib"):
                assert torch.equal(out[k], want0[k]), f"no-allocation render {k}"
        say("[tuning] queue blend: no-allocation renders equal the default dispatch")
    finally:
        r.close()
        renderer.set_tuning(**DEFAULT)
