"""Full-size parity of the HIP render path against the FP64 oracle, in the
launch configuration ``bench.py`` times (eager pair sizing, 16x16 tiles, the
workload's own camera and resolution).

At these sizes the oracle cannot emit and sort every pair (K reaches 10^9 at
4K), so it checks what it can compute one by one:

* every Gaussian's projection: integers and the centre bit-exact, the rest
  to float32 rounding (as in the small-scene tests);
* every tile's pair count, hence every tile offset, against the oracle's
  count of the rectangles covering the tile;
* the sorted lists of sampled tiles (corners, ragged edges, centre, the
  heaviest tiles and seeded random ones) against the oracle's per-tile list;
* every pixel of those tiles against the oracle's composite along that list,
  within 1e-4 on unambiguous pixels.

For BF16/FP16 attribute storage the bar above is taken against the
dequantised scene (what the kernel reads); the error against the FP64 render
of the float32 master scene is printed as max-abs and PSNR over the sampled
pixels, the precision report of the storage variants.
"""
import json
import math
import sys

import numpy as np
import pytest

import oracle
import scenes
from parity import check_projection, dequantised

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

TILE = 16
IMAGE_TOL = 1e-4
# Ambiguous pixels of the sampled tiles, as the oracle marks them for these
# seeded scenes: C3 fp32 2 of 4224, C3 bf16 8 of 3712, C5 bf16 17 of 3584,
# C5 fp16 11 of 3584; each case is capped at about twice its count.
MAX_AMBIGUOUS = {"C3/fp32": 4, "C3/bf16": 16, "C5/bf16": 34, "C5/fp16": 22}
# the batched workload's four views (1920x1080, 640x480, 1280x720, 256x256):
# 3, 0, 1 and 6 ambiguous sampled pixels
MAX_AMBIGUOUS_C4 = 12


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


def sample_tiles(counts: np.ndarray, tx: int, ty: int, n_random: int, seed: int) -> list:
    T = tx * ty
    picks = [0, tx - 1, T - tx, T - 1,                    # corners (the last row/column are ragged)
             (ty // 2) * tx + tx // 2,                    # centre
             (ty - 1) * tx + tx // 2, (ty // 2) * tx + tx - 1]   # ragged bottom row, ragged right column
    picks += [int(t) for t in np.argsort(-counts.astype(np.int64), kind="stable")[:3]]   # heaviest lists
    rng = np.random.default_rng(seed)
    picks += [int(t) for t in rng.integers(0, T, n_random)]
    seen, out = set(), []
    for t in picks:
        if t not in seen:
            seen.add(t)
            out.append(t)
    return out


def tile_pixels(t: int, tx: int, W: int, H: int):
    x0, y0 = (t % tx) * TILE, (t // tx) * TILE
    ys, xs = np.mgrid[y0:min(y0 + TILE, H), x0:min(x0 + TILE, W)]
    return xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)


def check_view_sampled(label: str, scene, ref_scene, cam, g: dict, offsets, values_dev, image, final_T, n_contrib,
                       n_random: int, seed: int, master_scene=None, max_ambiguous=None):
    """One view of a GPU render against the oracle, at any size: every
    Gaussian's projection, every tile's pair count, and the lists and pixels
    of sampled tiles.  ``g`` holds the view's projection (items of this view
    only, indices 0..n-1) and ``values_dev`` its list values as Gaussian
    indices; ``master_scene`` adds the error against the FP64 render of the
    float32 master scene."""
    W, H = cam["width"], cam["height"]
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    say(f"[fullsize] {label}: oracle projection")
    p = oracle.project(ref_scene, cam)
    amb = check_projection(g, p, label)
    # Gaussians whose 3-sigma radius sits on an integer boundary may bin
    # differently; every other rectangle is bit-exact, so the per-tile counts
    # and lists are compared where no such Gaussian differs
    differ = [int(i) for i in amb if not np.array_equal(g["rect"][i], p["rect"][:, i])]
    say(f"[fullsize] {label}: K={int(offsets[-1])} radius-ambiguous={len(amb)} differing={len(differ)}")
    counts = oracle.tile_counts(p).astype(np.int64)
    if not differ:
        want_off = np.concatenate([[0], np.cumsum(counts)])
        np.testing.assert_array_equal(offsets, want_off, err_msg=f"{label} tile offsets")
    else:
        bad = np.zeros(tx * ty, bool)
        for i in differ:
            for r in (g["rect"][i], p["rect"][:, i]):
                if r[2] > r[0] and r[3] > r[1]:
                    for yy in range(r[1], r[3]):
                        bad[yy * tx + r[0]: yy * tx + r[2]] = True
        np.testing.assert_array_equal(np.diff(offsets)[~bad], counts[~bad], err_msg=f"{label} tile counts")

    tiles = sample_tiles(counts, tx, ty, n_random, seed=seed)
    master = oracle.project(master_scene, cam) if master_scene is not None else None
    n_pix = n_amb = 0
    worst = 0.0
    se_master = 0.0
    max_master = 0.0
    for t in tiles:
        s, e = int(offsets[t]), int(offsets[t + 1])
        got = values_dev(s, e)
        want = oracle.tile_list(p, t)
        if not differ:
            np.testing.assert_array_equal(got, want, err_msg=f"{label} tile {t} list")
        else:   # every pair of the Gaussians binned alike, in order
            np.testing.assert_array_equal(got[~np.isin(got, differ)], want[~np.isin(want, differ)],
                                          err_msg=f"{label} tile {t} list")
        xs, ys = tile_pixels(t, tx, W, H)
        o5, marg = oracle.composite_pixels(p, xs, ys, want)
        amb_px = (marg[:, 0] < oracle.ALPHA_MARGIN) | (marg[:, 1] < oracle.T_MARGIN)
        gi = image[:, ys, xs].T.astype(np.float64)
        d = np.abs(gi - o5[:, :3]).max(axis=1)
        good = ~amb_px
        if good.any():
            worst = max(worst, float(d[good].max()))
            np.testing.assert_array_equal(n_contrib[ys, xs][good], o5[good, 4].astype(np.int64),
                                          err_msg=f"{label} tile {t} n_contrib")
            assert float(np.abs(final_T[ys, xs][good] - o5[good, 3]).max()) <= IMAGE_TOL, f"{label} tile {t} T"
        if amb_px.any():
            assert float(d[amb_px].max()) <= 0.01 * max(1.0, float(o5[:, :3].max())), f"{label} tile {t}"
        n_pix += len(xs)
        n_amb += int(amb_px.sum())
        if master is not None:
            mlist = oracle.tile_list(master, t)
            m5, _ = oracle.composite_pixels(master, xs, ys, mlist)
            dm = gi - m5[:, :3]
            se_master += float((dm ** 2).sum())
            max_master = max(max_master, float(np.abs(dm).max()))
    rep = dict(case=label, gaussians=int(scene["means"].shape[1]), width=W, height=H,
               pairs=int(offsets[-1]), tiles_sampled=len(tiles), pixels=n_pix, ambiguous=n_amb,
               max_abs_vs_oracle=worst)
    if master is not None:
        mse = se_master / (3 * n_pix)
        rep.update(max_abs_vs_fp64_master=max_master,
                   psnr_vs_fp64_master_db=(math.inf if mse == 0 else 10 * math.log10(1.0 / mse)))
    say("[fullsize] " + json.dumps(rep))
    assert worst <= IMAGE_TOL, f"{label}: max-abs {worst:.3e} on unambiguous sampled pixels"
    cap = MAX_AMBIGUOUS[label] if max_ambiguous is None else max_ambiguous
    assert n_amb <= cap, f"{label}: {n_amb} ambiguous of {n_pix}"
    return rep


def fullsize_case(renderer, workload: str, dtype: int, n_random: int):
    import torch
    import paper_2607_15951_amd as gs
    label = f"{workload}/{['fp32', 'bf16', 'fp16'][dtype]}"
    say(f"[fullsize] {label}: generating")
    scene = scenes.make_scene(workload)
    cam = scenes.make_cameras(workload)[0]
    W, H = cam["width"], cam["height"]
    dev = gs.scene_to_device(scene, dtype)
    say(f"[fullsize] {label}: GPU render n={scene['means'].shape[1]} {W}x{H}")
    out = renderer.render(dev, cam, W, H)
    torch.cuda.synchronize()
    lists = renderer.lists(keys=False)
    projg = renderer.projection()
    torch.cuda.synchronize()
    g = dict(splats=projg["splats"].cpu().numpy(),
             depth_key=projg["depth_key"].cpu().numpy().view(np.uint32),
             radius=projg["radius"].cpu().numpy(),
             tiles_touched=projg["tiles_touched"].cpu().numpy().view(np.uint32),
             rect=projg["rect"].cpu().numpy().view(np.uint16).astype(np.int32))
    offsets = lists["tile_offsets"].cpu().numpy().view(np.uint32).astype(np.int64)
    values = lists["values"]
    del dev
    return check_view_sampled(label, scene, dequantised(scene, dtype), cam, g, offsets,
                              lambda s, e: values[s:e].cpu().numpy().view(np.uint32),
                              out["image"].cpu().numpy(), out["final_T"].cpu().numpy(),
                              out["n_contrib"].cpu().numpy(), n_random,
                              seed=sum(map(ord, workload)) * 3 + dtype,
                              master_scene=scene if dtype else None)


def test_c4_batched_one_view_per_resolution(renderer):
    """The batched workload's scene (1M Gaussians, SH3) rendered in one
    gs_render_batched call from the first camera of each of its four
    resolutions: every view against the oracle like the single renders
    (projection, tile counts, sampled lists and pixels)."""
    import torch
    import paper_2607_15951_amd as gs
    scene = scenes.make_scene("C4")
    all_cams = scenes.make_cameras("C4")
    cams, seen = [], set()
    for c in all_cams:
        if (c["width"], c["height"]) not in seen:
            seen.add((c["width"], c["height"]))
            cams.append(c)
    assert len(cams) == 4
    n = scene["means"].shape[1]
    dev = gs.scene_to_device(scene, 0)
    say(f"[fullsize] C4: batched render of {len(cams)} views, n={n}")
    outs = renderer.render_batched(dev, cams)
    torch.cuda.synchronize()
    lists = renderer.lists(keys=False)
    projg = renderer.projection()
    torch.cuda.synchronize()
    offsets_all = lists["tile_offsets"].cpu().numpy().view(np.uint32).astype(np.int64)
    values = lists["values"]
    splats = projg["splats"].cpu().numpy()
    dk = projg["depth_key"].cpu().numpy().view(np.uint32)
    rad = projg["radius"].cpu().numpy()
    tt = projg["tiles_touched"].cpu().numpy().view(np.uint32)
    rect = projg["rect"].cpu().numpy().view(np.uint16).astype(np.int32)
    del dev
    tile_base = 0
    for v, (c, o) in enumerate(zip(cams, outs)):
        W, H = c["width"], c["height"]
        T = ((W + TILE - 1) // TILE) * ((H + TILE - 1) // TILE)
        sl = slice(v * n, (v + 1) * n)
        g = dict(splats=splats[sl], depth_key=dk[sl], radius=rad[sl], tiles_touched=tt[sl], rect=rect[sl])
        off = offsets_all[tile_base:tile_base + T + 1]
        base = int(off[0])

        def view_values(s, e, base=base, v=v):
            got = values[base + s:base + e].cpu().numpy().view(np.uint32).astype(np.int64) - v * n
            assert (got >= 0).all() and (got < n).all()
            return got.astype(np.uint32)

        check_view_sampled(f"C4/view{v} {W}x{H}", scene, scene, c, g, off - base, view_values,
                           o["image"].cpu().numpy(), o["final_T"].cpu().numpy(), o["n_contrib"].cpu().numpy(),
                           n_random=4, seed=400 + v, max_ambiguous=MAX_AMBIGUOUS_C4)
        tile_base += T


def test_c3_fp32_full_size(renderer):
    """The bench workload itself: 3M Gaussians, SH3, 1920x1080, fp32."""
    fullsize_case(renderer, "C3", 0, n_random=8)


def test_c3_bf16_full_size(renderer):
    fullsize_case(renderer, "C3", 1, n_random=6)


@pytest.mark.parametrize("dtype", [1, 2], ids=["bf16", "fp16"])
def test_c5_reduced_precision_4k(renderer, dtype):
    """6M Gaussians at 3840x2160 with BF16 / FP16 attribute storage."""
    fullsize_case(renderer, "C5", dtype, n_random=4)


# Whole images: every pixel of the 1080p frame against the oracle, rendered
# tile by tile (oracle.render_tiles: each tile's own list, no frame-wide sort).
# Ambiguous pixels of these frames as the oracle marks them: C3 fp32 4743 of
# 2073600 (2.3e-3: pixels composite more entries here than in the smaller
# scenes, so the transmittance bound reaches the threshold more often); the
# cap is about twice that.
WHOLE_AMBIGUOUS_FRAC = 5e-3


def whole_image_case(renderer, dtype: int):
    import torch
    import paper_2607_15951_amd as gs
    from parity import check_image, psnr
    label = f"C3/{['fp32', 'bf16', 'fp16'][dtype]} whole image"
    scene = scenes.make_scene("C3")
    cam = scenes.make_cameras("C3")[0]
    W, H = cam["width"], cam["height"]
    dev = gs.scene_to_device(scene, dtype)
    say(f"[whole] {label}: GPU render")
    out = renderer.render(dev, cam, W, H)
    torch.cuda.synchronize()
    g = dict(image=out["image"].cpu().numpy().astype(np.float64),
             final_T=out["final_T"].cpu().numpy().astype(np.float64), n_contrib=out["n_contrib"].cpu().numpy())
    del dev
    say(f"[whole] {label}: oracle, tile by tile")
    o = oracle.render_tiles(oracle.project(dequantised(scene, dtype), cam))
    stats = check_image(g, o, label, max_ambiguous_frac=WHOLE_AMBIGUOUS_FRAC)
    rep = dict(case=label, pixels=W * H, ambiguous=stats["ambiguous"], max_abs_vs_oracle=stats["max_abs"],
               psnr_vs_oracle_db=stats["psnr"])
    if dtype:
        say(f"[whole] {label}: FP64 render of the float32 master scene")
        m = oracle.render_tiles(oracle.project(scene, cam))
        rep.update(max_abs_vs_fp64_master=float(np.abs(g["image"] - m["image"]).max()),
                   psnr_vs_fp64_master_db=psnr(g["image"], m["image"]))
    say("[whole] " + json.dumps(rep))
    return rep


def test_c3_fp32_whole_image(renderer):
    """The bench frame, every pixel: 1e-4 against the FP64 oracle where no
    threshold decision is within float32 reach."""
    whole_image_case(renderer, 0)


@pytest.mark.parametrize("dtype", [1, 2], ids=["bf16", "fp16"])
def test_c3_reduced_precision_whole_image(renderer, dtype):
    """BF16 / FP16 attribute storage: parity with the oracle on the
    dequantised scene (every pixel), and the error of the stored precision
    against the FP64 render of the float32 master scene over the whole frame
    (BF16's 8-bit mantissa puts log-scales about 1% off, FP16's 11-bit one
    about 0.1%)."""
    rep = whole_image_case(renderer, dtype)
    assert rep["psnr_vs_fp64_master_db"] >= (50.0 if dtype == 1 else 60.0), rep
