"""Pins of the FP64 autograd oracle (``oracle.grad``) that the backward is
checked against, on the CPU.

* its forward equals the C oracle's render (image and final transmittance)
  to FP64 rounding, so it computes the same function of Eq. 1;
* a closed form: for one Gaussian and one pixel, C = a c + (1 - a) bg and
  dC/d(logit) = (c - bg) exp(p) s (1 - s) with s the sigmoid;
* its gradient equals central finite differences of the C oracle's render
  for sampled coordinates of every parameter group (means, log-scales,
  quaternions, opacity logits, SH coefficients), SH0 and SH3, with a
  background colour and a loss on the final transmittance.  Samples whose
  perturbation changes a discrete decision (a tile rectangle, an alpha
  threshold, a termination) are not smooth there and are redrawn.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.grad as og
import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def small_scene(kind: str):
    if kind == "sh0":
        sc = scenes.make_scene("C1", n=40, seed=71)
        cam = scenes.default_camera(40, 36)
    else:
        sc = scenes.make_scene("C2", n=50, seed=72, sh_degree=3)
        cam = scenes.look_at_camera([0.9, -0.5, -2.8], 44, 34)
    # larger footprints than the workload's (several pixels each), so that
    # every Gaussian reaches many pixels and lists overlap
    sc["log_scales"] = (sc["log_scales"] + np.float32(1.6)).astype(np.float32)
    return sc, cam


def weights(cam, seed):
    rng = np.random.default_rng(seed)
    H, W = cam["height"], cam["width"]
    return rng.uniform(-1.0, 1.0, (3, H, W)), rng.uniform(-1.0, 1.0, (H, W))


def c_loss(scene, cam, w_rgb, w_T, bg):
    r = oracle.render(scene, cam, background=bg)
    return float((w_rgb * r["image"]).sum() + (w_T * r["final_T"]).sum()), r


@pytest.mark.parametrize("kind", ["sh0", "sh3"])
def test_forward_equals_c_oracle(kind):
    sc, cam = small_scene(kind)
    bg = (0.2, 0.5, 0.1)
    ref = oracle.render(sc, cam, background=bg)
    assert ref["proj"]["visible"] > 10
    p = og.params_from_scene(sc, requires_grad=False)
    img, T = og.image_t(p, cam, bg, proj=ref["proj"])
    np.testing.assert_allclose(img.numpy(), ref["image"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(T.numpy(), ref["final_T"], rtol=0, atol=1e-12)


def test_single_gaussian_logit_closed_form():
    """One Gaussian in front of the camera, the pixel under its centre."""
    sc = dict(means=np.array([[0.013], [-0.021], [0.0]], np.float32),
              log_scales=np.full((3, 1), -1.0, np.float32),
              quats=np.array([[1.0], [0.0], [0.0], [0.0]], np.float32),
              opacity_logits=np.array([-0.4], np.float32),
              sh=np.array([[[0.3], [-0.2], [0.6]]], np.float32), sh_degree=0)
    cam = scenes.default_camera(32, 32)
    bg = (0.1, 0.7, 0.4)
    proj = oracle.project(sc, cam)
    H, W = 32, 32
    x, y = 16, 15
    w_rgb = np.zeros((3, H, W))
    w_rgb[0, y, x] = 1.0
    p = og.params_from_scene(sc)
    g = og.gradients(p, cam, w_rgb, np.zeros((H, W)), bg, proj=proj)
    u, v = proj["mean2d"][:, 0]
    A, B, Cc = proj["conic"][:, 0]
    dx, dy = u - x, v - y
    E = math.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
    s = 1.0 / (1.0 + math.exp(-float(sc["opacity_logits"][0])))
    assert s * E < 0.99 and s * E > 1.0 / 255.0
    want = (proj["rgb"][0, 0] - bg[0]) * E * s * (1.0 - s)
    assert abs(g["opacity_logits"][0] - want) <= 1e-12 * max(1.0, abs(want))
    # dC/d(sh_0 of red) = a Y_00 with a = s E
    want_sh = s * E * 0.5 * math.sqrt(1.0 / math.pi)
    assert abs(g["sh"][0, 0, 0] - want_sh) <= 1e-12


def perturbed(scene, group, idx, h):
    """Copies of the scene with one float32 coordinate moved by -h and +h;
    returns them and the exact float32 step between them."""
    lo, hi = dict(scene), dict(scene)
    a_lo, a_hi = scene[group].copy(), scene[group].copy()
    x = float(scene[group][idx])
    a_lo[idx] = np.float32(x - h)
    a_hi[idx] = np.float32(x + h)
    lo[group], hi[group] = a_lo, a_hi
    return lo, hi, float(a_hi[idx]) - float(a_lo[idx])


def decisions(scene, cam, w_rgb, w_T, bg, proj):
    p = og.params_from_scene(scene, requires_grad=False)
    _, masks = og.loss_t(p, cam, w_rgb, w_T, bg, proj=proj)
    return masks


def same_decisions(m1, m2):
    return all(torch.equal(m1[t], m2[t]) for t in m1)


@pytest.mark.parametrize("kind", ["sh0", "sh3"])
def test_gradient_matches_finite_differences(kind):
    sc, cam = small_scene(kind)
    bg = (0.3, 0.1, 0.6)
    w_rgb, w_T = weights(cam, seed=5 if kind == "sh0" else 6)
    base = oracle.project(sc, cam)
    p = og.params_from_scene(sc)
    g = og.gradients(p, cam, w_rgb, w_T, bg, proj=base)
    m0 = decisions(sc, cam, w_rgb, w_T, bg, base)
    vis = np.nonzero(base["tiles_touched"])[0]
    rng = np.random.default_rng(17 if kind == "sh0" else 18)
    h = 2e-4
    checked = {k: 0 for k in GROUPS}
    worst = 0.0
    tries = 0
    while min(checked.values()) < 4:
        tries += 1
        assert tries < 400, f"too few smooth samples: {checked}"
        group = GROUPS[int(rng.integers(0, len(GROUPS)))]
        if checked[group] >= 4:
            continue
        i = int(vis[rng.integers(0, len(vis))])
        shape = sc[group].shape
        if group == "opacity_logits":
            idx = (i,)
        elif group == "sh":
            idx = (int(rng.integers(0, shape[0])), int(rng.integers(0, 3)), i)
        else:
            idx = (int(rng.integers(0, shape[0])), i)
        lo, hi, step = perturbed(sc, group, idx, h)
        f_lo, r_lo = c_loss(lo, cam, w_rgb, w_T, bg)
        f_hi, r_hi = c_loss(hi, cam, w_rgb, w_T, bg)
        # smooth on the segment: same rectangles and the same composited sets
        if not (np.array_equal(r_lo["proj"]["rect"], base["rect"]) and
                np.array_equal(r_hi["proj"]["rect"], base["rect"])):
            continue
        if not (same_decisions(m0, decisions(lo, cam, w_rgb, w_T, bg, base)) and
                same_decisions(m0, decisions(hi, cam, w_rgb, w_T, bg, base))):
            continue
        fd = (f_hi - f_lo) / step
        ga = float(g[group][idx])
        # central differences carry O(h^2) truncation; the sum has ~1e3 terms
        tol = 2e-5 + 2e-4 * abs(ga)
        worst = max(worst, abs(fd - ga) / (1e-5 + abs(ga)))
        assert abs(fd - ga) <= tol, f"{kind} {group}{idx}: finite difference {fd:.9g} vs autograd {ga:.9g}"
        checked[group] += 1
    print(f"[oracle-grad] {kind}: worst relative |fd - autograd| = {worst:.2e}")


def test_culled_and_untouched_gaussians_have_zero_gradient():
    sc, cam = small_scene("sh0")
    # push two Gaussians behind the camera: culled, so no gradient
    sc["means"][2, :2] = np.float32(-5.0)
    bg = (0.0, 0.0, 0.0)
    w_rgb, w_T = weights(cam, seed=9)
    proj = oracle.project(sc, cam)
    assert proj["tiles_touched"][0] == 0 and proj["tiles_touched"][1] == 0
    p = og.params_from_scene(sc)
    g = og.gradients(p, cam, w_rgb, w_T, bg, proj=proj)
    for k in GROUPS:
        assert not np.any(g[k][..., :2]), k
