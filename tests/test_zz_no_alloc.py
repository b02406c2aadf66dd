"""gs_render_noalloc (the render for callers that cannot allocate) against
gs_render through the C ABI: two calls in a row, the second on a smaller
scene and image, each bit-identical to gs_render's image, final T and
n_contrib and reporting the same pair count; a scene too large for the
static scratch is refused before anything is written."""
import sys

import numpy as np
import pytest

import oracle
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


def outputs(W, H, fill):
    import torch
    return {"image": torch.full((3, H, W), fill, dtype=torch.float32, device="cuda"),
            "final_T": torch.full((H, W), fill, dtype=torch.float32, device="cuda"),
            "n_contrib": torch.full((H, W), -7, dtype=torch.int32, device="cuda")}


def test_noalloc_matches_render_on_two_calls(renderer):
    import torch
    import paper_2607_15951_amd as gs
    cases = [("C2-dist 40k 333x197", scenes.make_scene("C2", n=40_000, seed=21), scenes.default_camera(333, 197), 0),
             ("C1 1000 128x128", scenes.make_scene("C1"), scenes.default_camera(128, 128), None)]
    for label, sc, cam, cap in cases:
        W, H = cam["width"], cam["height"]
        dev = gs.scene_to_device(sc)
        want = renderer.render(dev, cam, W, H, out=outputs(W, H, 0.0))
        torch.cuda.synchronize()
        K = renderer.list_info()["num_pairs"]
        cap = K if cap is None else cap   # the second call: an exact capacity
        got = renderer.render_noalloc(dev, cam, W, H, outputs(W, H, -1.0), pair_capacity=cap)
        torch.cuda.synchronize()
        info = renderer.list_info()
        say(f"[noalloc] {label}: K={K} capacity={cap} noalloc K={info['num_pairs']}")
        assert info["num_pairs"] == K
        for k in ("image", "final_T", "n_contrib"):
            assert torch.equal(got[k], want[k]), f"{label}: {k} differs from gs_render"
        with pytest.raises(gs.GsError):
            renderer.lists()   # the lists of a no-allocation render are not kept
    # the last (smaller) one against the oracle as well
    o = oracle.render(sc, cam)
    amb = oracle.ambiguous_mask(o)
    d = np.abs(got["image"].cpu().numpy().astype(np.float64) - o["image"]).max(axis=0)
    assert float(d[~amb].max()) <= 1e-4


def test_noalloc_refuses_what_does_not_fit(renderer):
    """A million Gaussians need more than the scratch for their own buffers:
    refused with GS_ERR_CAPACITY before any launch (outputs untouched); an
    explicit capacity too large for the scratch likewise.  500k Gaussians
    fit, but not their 1.8e7 pairs: the derived capacity overflows on the
    device and gs_get_list_info reports it."""
    import torch
    import paper_2607_15951_amd as gs
    big = gs.scene_to_device(scenes.make_scene("C4"))
    out = outputs(256, 256, -3.0)
    with pytest.raises(gs.GsError) as e:
        renderer.render_noalloc(big, scenes.default_camera(256, 256), 256, 256, out)
    assert e.value.status == gs.GS_ERR_CAPACITY
    assert "scratch" in str(e.value)
    del big
    small = gs.scene_to_device(scenes.make_scene("C1"))
    out2 = outputs(128, 128, -3.0)
    with pytest.raises(gs.GsError) as e:
        renderer.render_noalloc(small, scenes.default_camera(128, 128), 128, 128, out2, pair_capacity=50_000_000)
    assert e.value.status == gs.GS_ERR_CAPACITY
    torch.cuda.synchronize()
    assert bool((out["image"] == -3.0).all()) and bool((out2["image"] == -3.0).all())
    mid = gs.scene_to_device(scenes.make_scene("C2"))
    out3 = outputs(1280, 720, -3.0)
    renderer.render_noalloc(mid, scenes.default_camera(1280, 720), 1280, 720, out3)
    with pytest.raises(gs.GsError) as e:
        renderer.list_info()
    assert e.value.status == gs.GS_ERR_CAPACITY
    # the context renders normally afterwards
    renderer.render_noalloc(small, scenes.default_camera(128, 128), 128, 128, out2)
    torch.cuda.synchronize()
    assert renderer.list_info()["num_pairs"] == 4517
    assert bool(torch.isfinite(out2["image"]).all())
