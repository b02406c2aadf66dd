"""GPU parity of the HIP render path against the FP64 oracle, through the C ABI.

Every test renders on the GPU via ``paper_2607_15951_amd.Renderer`` (which
calls ``gs_render``) and compares with ``oracle`` on the same seeded inputs:
bit-exact projection integers, keys, sorted lists and tile offsets; images
within 1e-4 max-abs on pixels whose threshold decisions are unambiguous.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import scenes
from parity import (batched_views, check_image, check_lists_full, check_projection, dequantised, gpu_render,
                    oracle_view_parity)

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


@pytest.fixture(scope="module")
def renderer():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_15951_amd as gs
    r = gs.Renderer(0)
    yield r
    r.close()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def full_parity(renderer, scene, cam, label, dtype=0, background=(0.0, 0.0, 0.0)):
    say(f"[parity] {label}: n={scene['means'].shape[1]} {cam['width']}x{cam['height']} dtype={dtype}")
    g = gpu_render(renderer, scene, cam, dtype=dtype, background=background)
    ref_scene = dequantised(scene, dtype)
    o = oracle.render(ref_scene, cam, background=background)
    amb = check_projection(g, o["proj"], label)
    removed = check_lists_full(g, o, label, exclude=amb)
    stats = check_image(g, o, label)
    say(f"[parity] {label}: K={len(o['keys'])} max_abs={stats['max_abs']:.2e} "
        f"ambiguous={stats['ambiguous']} psnr={stats['psnr']:.1f} radius_ambiguous={len(amb)} "
        f"pairs_removed={removed}")
    return g, o, stats


# --------------------------------------------------------------------------- workloads

def test_c1_full(renderer):
    sc = scenes.make_scene("C1")
    full_parity(renderer, sc, scenes.default_camera(128, 128), "C1 128x128")


def test_c1_ragged_tiles(renderer):
    sc = scenes.make_scene("C1", n=3000, seed=11)
    full_parity(renderer, sc, scenes.default_camera(200, 120), "C1-dist 200x120 ragged")


def test_mixture_sh3_medium(renderer):
    sc = scenes.make_scene("C2", n=40_000, seed=21)
    full_parity(renderer, sc, scenes.default_camera(333, 197), "C2-dist 40k 333x197")


def test_powerlaw_rotated_camera(renderer):
    sc = scenes.make_scene("C3", n=60_000, seed=31)
    cam = scenes.look_at_camera([1.2, -0.8, -2.7], 400, 240)
    full_parity(renderer, sc, cam, "C3-dist 60k rotated 400x240")


def test_c2_full_size(renderer):
    sc = scenes.make_scene("C2")
    full_parity(renderer, sc, scenes.default_camera(1280, 720), "C2 500k 1280x720")


def test_background_colour(renderer):
    sc = scenes.make_scene("C1", n=800, seed=5)
    full_parity(renderer, sc, scenes.default_camera(96, 80), "bg", background=(0.2, 0.5, 0.9))


@pytest.mark.parametrize("dtype", [1, 2], ids=["bf16", "fp16"])
def test_reduced_precision_storage(renderer, dtype):
    sc = scenes.make_scene("C2", n=30_000, seed=41)
    full_parity(renderer, sc, scenes.default_camera(256, 176), f"storage dtype {dtype}", dtype=dtype)


# --------------------------------------------------------------------------- closed forms on the GPU

def _tiny(means, log_scales, quats, logits, rgb):
    n = np.asarray(means).reshape(3, -1).shape[1]
    rgb = np.asarray(rgb, np.float64).reshape(3, n)
    return dict(means=np.ascontiguousarray(np.asarray(means, np.float32).reshape(3, n)),
                log_scales=np.ascontiguousarray(np.asarray(log_scales, np.float32).reshape(3, n)),
                quats=np.ascontiguousarray(np.asarray(quats, np.float32).reshape(4, n)),
                opacity_logits=np.ascontiguousarray(np.asarray(logits, np.float32).reshape(n)),
                sh=np.ascontiguousarray(((rgb - 0.5) / (0.5 / math.sqrt(math.pi)))[None].astype(np.float32)),
                sh_degree=0)


def test_single_gaussian_centre_is_colour_times_alpha(renderer):
    cam = scenes.default_camera(64, 64)
    sc = _tiny([0, 0, 0], [math.log(0.02)] * 3, [1, 0, 0, 0], [0.4], [[0.8], [0.4], [0.2]])
    g = gpu_render(renderer, sc, cam)
    alpha = 1 / (1 + math.exp(-float(np.float32(0.4))))
    rgb = sc["sh"][0, :, 0].astype(np.float64) * (0.5 / math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(g["image"][:, 32, 32], rgb * alpha, rtol=2e-6)
    np.testing.assert_allclose(g["final_T"][32, 32], 1 - alpha, rtol=2e-6)
    assert g["n_contrib"][32, 32] == 1


def test_termination_after_13_of_20(renderer):
    n = 20
    sc = _tiny([np.zeros(n), np.zeros(n), np.linspace(-0.5, 0.5, n)], np.full((3, n), -2.5),
               np.tile([[1], [0], [0], [0]], (1, n)), np.zeros(n), np.tile([[0.9], [0.5], [0.1]], (1, n)))
    g = gpu_render(renderer, sc, scenes.default_camera(32, 32))
    assert g["n_contrib"][16, 16] == 13
    assert g["final_T"][16, 16] == 2.0 ** -13
    T = g["final_T"]
    assert (T >= 1e-4).all() and (T <= 1).all()


# --------------------------------------------------------------------------- edge cases

def test_empty_scene(renderer):
    import torch
    import paper_2607_15951_amd as gs
    dev = {"sh_degree": 0, "attr_dtype": 0}
    for k, shape in (("means", (3, 0)), ("log_scales", (3, 0)), ("quats", (4, 0)), ("opacity_logits", (0,)),
                     ("sh", (1, 3, 0))):
        dev[k] = torch.zeros(shape, dtype=torch.float32, device="cuda")
    out = renderer.render(dev, scenes.default_camera(40, 24), 40, 24, background=(0.25, 0.5, 0.75))
    torch.cuda.synchronize()
    img = out["image"].cpu().numpy()
    np.testing.assert_array_equal(img, np.broadcast_to(np.array([0.25, 0.5, 0.75], np.float32)[:, None, None],
                                                       img.shape))
    assert (out["final_T"].cpu().numpy() == 1).all()
    info = renderer.list_info()
    assert info["num_pairs"] == 0 and info["n_visible"] == 0


def test_everything_culled(renderer):
    sc = scenes.make_scene("C1", n=500, seed=3)
    sc["means"][2] = np.float32(-5.0)   # all behind the camera
    g = gpu_render(renderer, sc, scenes.default_camera(64, 64))
    assert g["num_pairs"] == 0 and g["n_visible"] == 0
    assert (g["image"] == 0).all() and (g["final_T"] == 1).all()


def test_one_pixel_image(renderer):
    sc = scenes.make_scene("C1", n=2000, seed=4)
    full_parity(renderer, sc, scenes.default_camera(1, 1), "1x1")


def test_bad_gaussians_cull_only_themselves(renderer):
    sc = scenes.make_scene("C1", n=400, seed=9)
    cam = scenes.default_camera(96, 64)
    bad = dict(sc)
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    bad["means"][0, 10] = np.nan
    bad["quats"][:, 20] = 0.0
    g_bad = gpu_render(renderer, bad, cam)
    keep = np.setdiff1d(np.arange(400), [10, 20])
    ok = {k: (np.ascontiguousarray(v[..., keep]) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    g_ok = gpu_render(renderer, ok, cam)
    assert g_bad["tiles_touched"][10] == 0 and g_bad["tiles_touched"][20] == 0
    np.testing.assert_array_equal(g_bad["image"], g_ok["image"])
    o = oracle.render(bad, cam)
    check_projection(g_bad, o["proj"], "bad data")
    check_lists_full(g_bad, o, "bad data")


def test_huge_gaussian_covers_every_tile(renderer):
    sc = scenes.make_scene("C1", n=200, seed=12)
    sc["log_scales"][:, 0] = np.float32(0.5)
    sc["means"][:, 0] = 0.0
    full_parity(renderer, sc, scenes.default_camera(150, 90), "huge")


def test_grid_wider_than_packed_rectangles(renderer):
    """263 tile columns: past the 255 of the rectangles packed into one word,
    so the depth sort carries no rectangles and the row counts gather them."""
    sc = scenes.make_scene("C2", n=20_000, seed=91)
    full_parity(renderer, sc, scenes.default_camera(4200, 120), "4200x120 (263 tile columns)")


@pytest.mark.parametrize("size", [(32768, 32), (32, 32768)], ids=["max_width", "max_height"])
def test_largest_image_dimensions(renderer, size):
    """The widest and the tallest image the library accepts: 2048 tile
    columns, or 2048 tile rows (the LDS difference arrays of the binning are
    sized by them)."""
    sc = scenes.make_scene("C1", n=400, seed=92)
    full_parity(renderer, sc, scenes.default_camera(*size), f"{size[0]}x{size[1]}")


def test_more_than_2_32_pairs_is_refused_before_the_pair_buffers(renderer):
    """4.9e9 (Gaussian, tile) pairs: 600k Gaussians that each cover all 8160
    tiles of a 1080p image.  Pair offsets are 32-bit, so the eager render
    stops after the row counts with GS_ERR_CAPACITY: no output written, and
    no pair buffer allocated (the device's free memory does not drop by the
    20 GB it would take)."""
    import torch
    import paper_2607_15951_amd as gs
    n = 600_000
    rng = np.random.default_rng(14)
    sc = _tiny(rng.uniform(-0.05, 0.05, (3, n)), np.full((3, n), 0.5), np.tile([[1], [0], [0], [0]], (1, n)),
               np.zeros(n), rng.uniform(0, 1, (3, n)))
    cam = scenes.default_camera(1920, 1080)
    dev = gs.scene_to_device(sc)
    out = {"image": torch.full((3, 1080, 1920), -2.0, device="cuda"),
           "final_T": torch.full((1080, 1920), -2.0, device="cuda"),
           "n_contrib": torch.full((1080, 1920), -2, dtype=torch.int32, device="cuda")}
    r = gs.Renderer(0)
    try:
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        with pytest.raises(gs.GsError) as e:
            r.render(dev, cam, 1920, 1080, out=out)
        assert e.value.status == gs.GS_ERR_CAPACITY, str(e.value)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        say(f"[capacity] {e.value}; device memory taken by the attempt: {(free0 - free1) / 2**30:.2f} GiB")
        assert free0 - free1 < 4 * 2**30
        assert bool((out["image"] == -2.0).all()) and bool((out["final_T"] == -2.0).all())
        assert bool((out["n_contrib"] == -2).all())
        # the context renders normally afterwards
        small = gs.scene_to_device(scenes.make_scene("C1"))
        r.render(small, scenes.default_camera(128, 128), 128, 128)
        assert r.list_info()["num_pairs"] == 4517
    finally:
        r.close()


def test_pair_capacity_mode(renderer):
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C1", n=1500, seed=13)
    cam = scenes.default_camera(128, 96)
    ref = gpu_render(renderer, sc, cam)
    K = ref["num_pairs"]
    same = gpu_render(renderer, sc, cam, pair_capacity=K)
    np.testing.assert_array_equal(same["image"], ref["image"])
    np.testing.assert_array_equal(same["values"], ref["values"])
    with pytest.raises(gs.GsError) as e:
        gpu_render(renderer, sc, cam, pair_capacity=K - 1)
    assert e.value.status == gs.GS_ERR_CAPACITY
    again = gpu_render(renderer, sc, cam)   # context still usable
    np.testing.assert_array_equal(again["image"], ref["image"])


def test_context_reuse_across_sizes(renderer):
    a = scenes.make_scene("C2", n=20_000, seed=51)
    b = scenes.make_scene("C1", n=300, seed=52)
    ca, cb = scenes.default_camera(300, 200), scenes.default_camera(64, 48)
    ga1 = gpu_render(renderer, a, ca)
    gb = gpu_render(renderer, b, cb)
    ga2 = gpu_render(renderer, a, ca)
    np.testing.assert_array_equal(ga1["image"], ga2["image"])
    np.testing.assert_array_equal(ga1["values"], ga2["values"])
    o = oracle.render(b, cb)
    check_lists_full(gb, o, "small after large")


def test_row_entries_outgrowing_the_last_render():
    """An eager render scatters its row entries into the buffer an earlier
    render left while the host reads this frame's sizes, and scatters them
    again into a grown buffer when they do not fit.  A large render after a
    small one on the same context must equal the same render on a fresh
    context, and the oracle's lists."""
    import paper_2607_15951_amd as gs
    small = scenes.make_scene("C2", n=2_000, seed=71)
    big = scenes.make_scene("C2", n=40_000, seed=72)
    cam = scenes.default_camera(333, 197)
    r1, r2 = gs.Renderer(0), gs.Renderer(0)
    try:
        gpu_render(r1, small, cam)
        r_small = r1.list_info()["num_row_entries"]
        g1 = gpu_render(r1, big, cam)
        r_big = r1.list_info()["num_row_entries"]
        # the second render's entries exceed the buffer sized for the first
        # (sizes grow by a quarter)
        assert r_big > 2 * r_small, (r_small, r_big)
        g2 = gpu_render(r2, big, cam)
        for k in ("image", "final_T", "n_contrib", "values", "tile_offsets", "keys"):
            np.testing.assert_array_equal(g1[k], g2[k])
        o = oracle.render(big, cam)
        amb = check_projection(g1, o["proj"], "row entries outgrowing the last render")
        check_lists_full(g1, o, "row entries outgrowing the last render", exclude=amb)
        g3 = gpu_render(r1, big, cam)   # the same frame again: its entries fit the grown buffer
        np.testing.assert_array_equal(g3["values"], g2["values"])
    finally:
        r1.close()
        r2.close()


def test_module_render_from_rows(renderer):
    """The module-level render() of a scene given as per-Gaussian rows
    ([N, C], transposed once by scene_from_rows) equals Renderer.render of
    the channel-major scene, image and lists."""
    import torch
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=5_000, seed=81)
    cam = scenes.default_camera(200, 120)
    dev = gs.scene_to_device(sc)
    rows = gs.scene_from_rows(dev["means"].t(), dev["log_scales"].t(), dev["quats"].t(), dev["opacity_logits"],
                              dev["sh"].permute(2, 0, 1))
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        assert torch.equal(rows[k], dev[k]), k
    img, lists = gs.render(rows, cam, (cam["width"], cam["height"]), keys=True)
    torch.cuda.synchronize()
    ref = gpu_render(renderer, sc, cam)
    np.testing.assert_array_equal(img.cpu().numpy().astype(np.float64), ref["image"])
    np.testing.assert_array_equal(lists["values"].cpu().numpy().view(np.uint32), ref["values"])
    np.testing.assert_array_equal(lists["tile_offsets"].cpu().numpy().view(np.uint32), ref["tile_offsets"])
    np.testing.assert_array_equal(lists["keys"].cpu().numpy().view(np.uint64), ref["keys"])
    assert lists["num_pairs"] == ref["num_pairs"]


def test_permutation_and_repeat_determinism(renderer):
    sc = scenes.make_scene("C2", n=10_000, seed=61)
    cam = scenes.default_camera(200, 150)
    g1 = gpu_render(renderer, sc, cam)
    g2 = gpu_render(renderer, sc, cam)
    for k in ("image", "final_T", "n_contrib", "values", "keys"):
        np.testing.assert_array_equal(g1[k], g2[k])


def test_traced_render_is_identical_and_consistent(renderer):
    """The work-counting blend variant renders the same image as the timed one,
    and its per-tile records are consistent with the lists and each other."""
    import torch
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=20_000, seed=71)
    cam = scenes.default_camera(300, 200)
    g0 = gpu_render(renderer, sc, cam)
    renderer.set_profiling(stages=True, blend_work=True)
    try:
        g1 = gpu_render(renderer, sc, cam)
        stats = renderer.blend_stats()
        tw = renderer.blend_tile_work().astype(np.int64)
        st = renderer.stage_times()
    finally:
        renderer.set_profiling(stages=False)
    for k in ("image", "final_T", "n_contrib", "values"):
        np.testing.assert_array_equal(g0[k], g1[k])
    T = ((300 + 15) // 16) * ((200 + 15) // 16)
    assert tw.shape == (T, 6)
    lens = np.diff(g1["tile_offsets"].astype(np.int64))
    assert (tw[:, 1] >= tw[:, 0]).all()
    assert (tw[:, 2] <= lens).all() and (tw[:, 5] <= tw[:, 4]).all()
    assert stats["staged"] == tw[:, 2].sum() and stats["lane_evaluations"] == 64 * tw[:, 3].sum()
    assert stats["evaluations"] == tw[:, 4].sum() and stats["composited"] == tw[:, 5].sum()
    # every composited evaluation is one a wave executed
    assert stats["composited"] <= stats["lane_evaluations"]
    # a pixel's last contributor was composited: n_contrib > 0 implies one composite
    assert stats["composited"] >= int((g1["n_contrib"] > 0).sum())
    assert all(v >= 0 for v in st.values())
    # a render without the flag is not counted
    gpu_render(renderer, sc, cam)
    with pytest.raises(gs.GsError):
        renderer.blend_stats()


def test_batched_views_equal_single_renders(renderer):
    """gs_render_batched over views of mixed (and ragged) sizes returns, for
    every view, the image, transmittance, n_contrib and per-tile lists of
    that view rendered alone; the lists of view v hold items v * n + i."""
    import torch
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=30_000, seed=81)
    n = sc["means"].shape[1]
    rng = np.random.default_rng(82)
    sizes = [(256, 256), (200, 120), (640, 480), (333, 197), (64, 48)]
    cams = []
    for (w, h) in sizes:
        e = rng.standard_normal(3)
        cams.append(scenes.look_at_camera(3.5 * e / np.linalg.norm(e), w, h))
    cams.append(scenes.default_camera(300, 200))
    singles = [gpu_render(renderer, sc, c) for c in cams]
    dev = gs.scene_to_device(sc)
    outs = renderer.render_batched(dev, cams)
    torch.cuda.synchronize()
    lists = renderer.lists(keys=True)
    info = renderer.list_info()
    assert info["num_views"] == len(cams)
    values = lists["values"].cpu().numpy().view(np.uint32)
    offsets = lists["tile_offsets"].cpu().numpy().view(np.uint32).astype(np.int64)
    keys = lists["keys"].cpu().numpy().view(np.uint64)
    tile_base = 0
    for v, (c, o, g) in enumerate(zip(cams, outs, singles)):
        say(f"[batched] view {v}: {c['width']}x{c['height']} K={g['num_pairs']}")
        np.testing.assert_array_equal(o["image"].cpu().numpy(), g["image"].astype(np.float32))
        np.testing.assert_array_equal(o["final_T"].cpu().numpy(), g["final_T"].astype(np.float32))
        np.testing.assert_array_equal(o["n_contrib"].cpu().numpy(), g["n_contrib"])
        T = ((c["width"] + 15) // 16) * ((c["height"] + 15) // 16)
        off = offsets[tile_base:tile_base + T + 1]
        np.testing.assert_array_equal(off - off[0], g["tile_offsets"].astype(np.int64))
        got = values[off[0]:off[-1]]
        np.testing.assert_array_equal(got, g["values"].astype(np.uint64) + np.uint64(v * n))
        # keys carry the global tile index and the depth bits of the item
        want_keys = g["keys"] + (np.uint64(tile_base) << np.uint64(32))
        np.testing.assert_array_equal(keys[off[0]:off[-1]], want_keys)
        tile_base += T
    assert tile_base == info["num_tiles"]
    assert info["num_pairs"] == sum(g["num_pairs"] for g in singles)
    # and every view against the oracle directly
    for v, (c, gv) in enumerate(zip(cams, batched_views(renderer, outs, cams, n))):
        st = oracle_view_parity(gv, sc, c, f"batched view {v}")
        say(f"[batched] view {v} vs oracle: {st}")


def test_batched_rejects_bad_views(renderer):
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C1", n=100, seed=83)
    dev = gs.scene_to_device(sc)
    good = scenes.default_camera(64, 64)
    bad = dict(good)
    bad["fx"] = np.float32(float("nan"))
    with pytest.raises(gs.GsError):
        renderer.render_batched(dev, [good, bad])
    with pytest.raises(gs.GsError):
        renderer.render_batched(dev, [])
    # the context still renders afterwards
    out = renderer.render_batched(dev, [good])
    assert out[0]["image"].shape == (3, 64, 64)


def test_graph_replays_match_eager_batched_render(renderer):
    """A captured batched render (gs_graph_*) replayed several times, with
    eager work and synchronisations between replays, returns the eager
    batched render's images every time; new cameras of the same sizes take
    effect on the next replay."""
    import torch
    import paper_2607_15951_amd as gs
    sc = scenes.make_scene("C2", n=20_000, seed=91)
    dev = gs.scene_to_device(sc)

    def cams_at(seed_shift):
        out = []
        for k, (w, h) in enumerate([(320, 240), (200, 120), (256, 256)]):
            e = np.random.default_rng(1000 * seed_shift + k).standard_normal(3)
            out.append(scenes.look_at_camera(3.5 * e / np.linalg.norm(e), w, h))
        return out

    cams = cams_at(1)
    ref = gs.Renderer(0)   # eager reference on its own context
    try:
        want = [{k: v.clone() for k, v in o.items()} for o in ref.render_batched(dev, cams)]
        K = ref.list_info()["num_pairs"]
        cams2 = cams_at(2)
        want2 = [{k: v.clone() for k, v in o.items()} for o in ref.render_batched(dev, cams2)]
        K2 = ref.list_info()["num_pairs"]
    finally:
        ref.close()
    cap = int(1.5 * max(K, K2)) + 64
    r = gs.Renderer(0)
    try:
        gr = r.graph(dev, cams, pair_capacity=cap)
        with pytest.raises(gs.GsError):   # the context belongs to the graph
            r.render(dev, cams[0], cams[0]["width"], cams[0]["height"])
        for rep in range(3):
            for o in gr.outs:
                o["image"].fill_(-1.0)
            torch.cuda.synchronize()
            gr.launch()
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()   # eager work between replays
            assert r.list_info()["num_pairs"] == K
            for o, w in zip(gr.outs, want):
                for k in ("image", "final_T", "n_contrib"):
                    assert torch.equal(o[k], w[k]), f"replay {rep} {k}"
        # the replayed views against the oracle directly
        n = sc["means"].shape[1]
        for v, (c, gv) in enumerate(zip(cams, batched_views(r, gr.outs, cams, n))):
            say(f"[graph] view {v} vs oracle: {oracle_view_parity(gv, sc, c, f'graph view {v}')}")
        gr.set_views(cams2)
        gr.launch()
        torch.cuda.synchronize()
        assert r.list_info()["num_pairs"] == K2
        for o, w in zip(gr.outs, want2):
            for k in ("image", "final_T", "n_contrib"):
                assert torch.equal(o[k], w[k]), f"new views {k}"
        for v, (c, gv) in enumerate(zip(cams2, batched_views(r, gr.outs, cams2, n))):
            say(f"[graph] new view {v} vs oracle: {oracle_view_parity(gv, sc, c, f'graph new view {v}')}")
        gr.close()
        # the context renders eagerly again once the graph is gone
        r.render(dev, cams[0], cams[0]["width"], cams[0]["height"])
    finally:
        r.close()
