"""Pins of the FP64 oracle against things other than itself.

Every check here compares the oracle with a library routine, a closed form, an
invariant or a brute-force computation, so that a dropped term, a wrong sign or
index, or a transposed operand anywhere in ``oracle/gs_oracle.c`` fails at
least one test.  No GPU involved.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
import scipy.special as sps

import oracle
import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")


def tiny_scene(means, log_scales, quats, logits, rgb=None, sh=None):
    means = np.asarray(means, np.float32).reshape(3, -1)
    n = means.shape[1]
    if sh is None:
        rgb = np.asarray(rgb, np.float64).reshape(3, n)
        sh = ((rgb - 0.5) / (0.5 / math.sqrt(math.pi)))[None]
        deg = 0
    else:
        deg = int(round(math.sqrt(sh.shape[0]))) - 1
    return dict(means=np.ascontiguousarray(means),
                log_scales=np.ascontiguousarray(np.asarray(log_scales, np.float32).reshape(3, n)),
                quats=np.ascontiguousarray(np.asarray(quats, np.float32).reshape(4, n)),
                opacity_logits=np.ascontiguousarray(np.asarray(logits, np.float32).reshape(n)),
                sh=np.ascontiguousarray(np.asarray(sh, np.float32)), sh_degree=deg)


def rotated_camera(W=64, H=48):
    cam = scenes.look_at_camera([1.3, -0.7, -2.6], W, H)
    return cam


# --------------------------------------------------------------------------- rotation, covariance

def test_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    cam = scenes.default_camera(64, 64)
    for _ in range(50):
        q = rng.standard_normal(4) * rng.uniform(0.2, 3.0)   # not unit: the oracle normalises
        g = oracle.debug_geometry(cam, [0.1, -0.2, 0.3], [-3, -3, -3], q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy is scalar-last
        np.testing.assert_allclose(g["Rq"], ref, atol=1e-14)
        g2 = oracle.debug_geometry(cam, [0.1, -0.2, 0.3], [-3, -3, -3], -q)
        np.testing.assert_allclose(g2["Rq"], g["Rq"], atol=1e-15)


def test_covariance_eigenvalues_and_axes():
    rng = np.random.default_rng(1)
    cam = scenes.default_camera(64, 64)
    for _ in range(50):
        q = rng.standard_normal(4)
        ls = rng.normal(-2.0, 1.0, 3)
        g = oracle.debug_geometry(cam, [0.0, 0.0, 0.0], ls, q)
        np.testing.assert_allclose(np.linalg.eigvalsh(g["Sigma"]), np.sort(np.exp(2 * ls)), rtol=1e-10)
        # each rotated axis is an eigenvector with eigenvalue exp(2 s_k)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        for k in range(3):
            np.testing.assert_allclose(g["Sigma"] @ R[:, k], math.exp(2 * ls[k]) * R[:, k],
                                       atol=1e-12 * math.exp(2 * ls.max()))


def test_jacobian_central_difference():
    cam = rotated_camera()
    f = float(cam["fx"])
    rng = np.random.default_rng(2)
    for _ in range(20):
        mu = rng.uniform(-0.3, 0.3, 3)
        g = oracle.debug_geometry(cam, mu, [-3, -3, -3], [1, 0, 0, 0])
        t = g["tcam"]
        # inside the guard band the clamp is inactive
        assert abs(t[0] / t[2]) < 1.3 * 0.5 * cam["width"] / f
        pi = lambda p: np.array([f * p[0] / p[2], f * p[1] / p[2]])
        h = 1e-6
        num = np.stack([(pi(t + h * e) - pi(t - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(g["J"], num, rtol=1e-7, atol=1e-6)


def test_jacobian_guard_band_clamps():
    cam = scenes.default_camera(64, 64)
    f = float(cam["fx"])
    lim = 1.3 * 32 / f
    g = oracle.debug_geometry(cam, [3.0, 0.0, 0.0], [-3, -3, -3], [1, 0, 0, 0])   # x/z = 1 > lim
    t = g["tcam"]
    assert t[0] / t[2] > lim
    np.testing.assert_allclose(g["J"][0, 2], -f * (lim * t[2]) / t[2] ** 2, rtol=1e-14)


def test_projected_covariance_monte_carlo():
    """Sample the 3D Gaussian, push samples through the camera and the
    perspective map: their covariance is J W Sigma W^T J^T (linearisation of
    a small Gaussian), i.e. the oracle's cov2d minus the 0.3 low-pass."""
    cam = rotated_camera(640, 480)
    rng = np.random.default_rng(3)
    mu = np.array([0.15, -0.1, 0.2])
    ls = np.array([-6.0, -6.8, -7.5])
    q = np.array([0.8, 0.3, -0.4, 0.2])
    g = oracle.debug_geometry(cam, mu, ls, q)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    m = 400_000
    X = mu[:, None] + R @ (np.exp(ls)[:, None] * rng.standard_normal((3, m)))
    Rc = np.asarray(cam["R"], np.float64)
    tc = np.asarray(cam["t"], np.float64)
    P = Rc @ X + tc[:, None]
    f = float(cam["fx"])
    uv = np.stack([f * P[0] / P[2], f * P[1] / P[2]])
    emp = np.cov(uv)
    a, b, c = g["cov2d"]
    ref = np.array([[a - 0.3, b], [b, c - 0.3]])
    np.testing.assert_allclose(emp, ref, rtol=0.02, atol=0.02 * np.abs(ref).max())
    # the 2D mean is the image of the centre
    np.testing.assert_allclose([g["u"], g["v"]],
                               [f * g["tcam"][0] / g["tcam"][2] + cam["cx"],
                                f * g["tcam"][1] / g["tcam"][2] + cam["cy"]], rtol=1e-13)


def test_conic_eigen_radius():
    rng = np.random.default_rng(4)
    cam = rotated_camera(320, 240)
    for _ in range(50):
        g = oracle.debug_geometry(cam, rng.uniform(-0.5, 0.5, 3), rng.normal(-3, 1, 3),
                                  rng.standard_normal(4))
        a, b, c = g["cov2d"]
        S = np.array([[a, b], [b, c]])
        A, B, Cc = g["conic"]
        np.testing.assert_allclose(np.array([[A, B], [B, Cc]]) @ S, np.eye(2), atol=1e-9)
        lam = np.linalg.eigvalsh(S).max()
        np.testing.assert_allclose(g["lambda_max"], lam, rtol=1e-10)
        assert g["radius"] == math.ceil(3 * math.sqrt(lam))


# --------------------------------------------------------------------------- colour

def real_sh_scipy(d):
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = []
    for l in range(4):
        for m in range(-l, l + 1):
            if m < 0:
                out.append(math.sqrt(2) * sps.sph_harm_y(l, -m, theta, phi).imag)
            elif m == 0:
                out.append(sps.sph_harm_y(l, 0, theta, phi).real)
            else:
                out.append(math.sqrt(2) * sps.sph_harm_y(l, m, theta, phi).real)
    return np.array(out)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(5)
    for _ in range(200):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        np.testing.assert_allclose(oracle.sh_basis(d), real_sh_scipy(d), atol=1e-13)


def test_sh_basis_orthonormal_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 exactly
    zs, wz = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * 2 * np.pi / 24
    G = np.zeros((16, 16))
    for z, w in zip(zs, wz):
        s = math.sqrt(1 - z * z)
        for p in phis:
            Y = oracle.sh_basis([s * math.cos(p), s * math.sin(p), z])
            G += w * (2 * np.pi / 24) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_colour_degree0_reproduces_rgb_and_clamps():
    rgb = np.array([[0.25, 0.0], [0.5, 1.0], [0.75, 0.3]])
    sc = tiny_scene([[0, 0.1], [0, 0], [0, 0]], np.full((3, 2), -3.0), [[1, 1], [0, 0], [0, 0], [0, 0]],
                    [0, 0], rgb=rgb)
    p = oracle.project(sc, scenes.default_camera(32, 32))
    np.testing.assert_allclose(p["rgb"], rgb, atol=1e-7)   # float32 storage of the coefficient
    sc["sh"][0, 0, 1] = -5.0
    p = oracle.project(sc, scenes.default_camera(32, 32))
    assert p["rgb"][0, 1] == 0.0


def test_colour_view_dependent_degree1():
    # one Gaussian at the origin seen from the default camera: direction (0,0,1)
    sh = np.zeros((4, 3, 1), np.float32)
    sh[2, :, 0] = [0.5, -0.25, 0.1]   # Y_{1,0} = c1 z
    sc = tiny_scene([0, 0, 0], [-3, -3, -3], [1, 0, 0, 0], [0], sh=sh)
    p = oracle.project(sc, scenes.default_camera(32, 32))
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(p["rgb"][:, 0], np.maximum(0, np.array([0.5, -0.25, 0.1]) * c1 + 0.5),
                               rtol=1e-7)


# --------------------------------------------------------------------------- closed forms

def _iso_setup(W=64, H=64, sigma_w=0.02, logit=0.4, rgb=(0.8, 0.4, 0.2)):
    sc = tiny_scene([0, 0, 0], [math.log(sigma_w)] * 3, [1, 0, 0, 0], [logit],
                    rgb=np.array(rgb)[:, None])
    cam = scenes.default_camera(W, H)
    return sc, cam


def test_single_isotropic_gaussian_closed_form():
    sc, cam = _iso_setup()
    res = oracle.render(sc, cam)
    f = float(cam["fx"])
    sw = float(np.float32(math.log(0.02)))
    v = (f * math.exp(sw) / 3) ** 2 + 0.3
    alpha = 1 / (1 + math.exp(-float(np.float32(0.4))))
    rgb = np.array([0.8, 0.4, 0.2])
    r = math.ceil(3 * math.sqrt(v))
    assert res["proj"]["radius"][0] == r
    # centre pixel: colour * alpha, T = 1 - alpha
    np.testing.assert_allclose(res["image"][:, 32, 32], rgb * alpha, rtol=1e-6)
    np.testing.assert_allclose(res["final_T"][32, 32], 1 - alpha, rtol=1e-12)
    # every pixel: the closed form, or untouched when alpha < 1/255
    ys, xs = np.mgrid[0:64, 0:64]
    a = alpha * np.exp(-((xs - 32.0) ** 2 + (ys - 32.0) ** 2) / (2 * v))
    a = np.minimum(a, 0.99)
    a = np.where(a < 1 / 255, 0.0, a)
    np.testing.assert_allclose(res["image"], rgb[:, None, None] * a[None], atol=2e-7)
    np.testing.assert_allclose(res["final_T"], 1 - a, atol=1e-12)


def test_two_on_axis_gaussians_closed_form():
    rgb = np.array([[1.0, 0.0], [0.0, 1.0], [0.2, 0.6]])
    logits = [0.3, -0.5]
    cam = scenes.default_camera(32, 32)
    for zs in ([0.0, 0.5], [0.5, 0.0]):
        sc = tiny_scene([[0, 0], [0, 0], zs], np.full((3, 2), -2.5), [[1, 1], [0, 0], [0, 0], [0, 0]],
                        logits, rgb=rgb)
        res = oracle.render(sc, cam)
        a = 1 / (1 + np.exp(-np.asarray(logits, np.float32).astype(np.float64)))
        front, back = (0, 1) if zs[0] < zs[1] else (1, 0)
        ref = rgb[:, front] * a[front] + rgb[:, back] * a[back] * (1 - a[front])
        # rgb passes through a float32 SH coefficient: 1e-7 relative
        np.testing.assert_allclose(res["image"][:, 16, 16], ref, atol=2e-7)
        assert res["n_contrib"][16, 16] == 2


def test_termination_closed_form():
    n = 20
    zs = np.linspace(-0.5, 0.5, n)
    rgb = np.tile(np.array([[0.9], [0.5], [0.1]]), (1, n))
    sc = tiny_scene([np.zeros(n), np.zeros(n), zs], np.full((3, n), -2.5),
                    np.tile([[1], [0], [0], [0]], (1, n)), np.zeros(n), rgb=rgb)
    res = oracle.render(sc, scenes.default_camera(32, 32))
    assert res["n_contrib"][16, 16] == 13
    np.testing.assert_allclose(res["final_T"][16, 16], 2.0 ** -13, rtol=0, atol=0)
    np.testing.assert_allclose(res["image"][:, 16, 16], rgb[:, 0] * (1 - 2.0 ** -13), atol=2e-7)


# --------------------------------------------------------------------------- invariants

def random_small(seed, n=40, W=48, H=40, logit_shift=0.0, deg=0):
    sc = scenes.make_scene("C1", n=n, seed=seed, sh_degree=deg)
    sc["means"] *= np.float32(0.6)
    sc["opacity_logits"] += np.float32(logit_shift)
    return sc, scenes.default_camera(W, H)


@pytest.mark.parametrize("seed", range(6))
def test_transmittance_bounds_and_white_scene(seed):
    sc, cam = random_small(seed, logit_shift=1.5)
    # all-white colours: the image equals 1 - T (weights telescope)
    sc["sh"][:] = np.float32(0.5 / (0.5 / math.sqrt(math.pi)))
    res = oracle.render(sc, cam)
    T = res["final_T"]
    assert (T >= 1e-4).all() and (T <= 1).all()
    np.testing.assert_allclose(res["image"], np.broadcast_to(1 - T, res["image"].shape), atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_permutation_invariance(seed):
    sc, cam = random_small(seed, n=60, deg=1)
    res = oracle.render(sc, cam)
    perm = np.random.default_rng(99 + seed).permutation(60)
    sc2 = {k: (np.ascontiguousarray(v[..., perm]) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    res2 = oracle.render(sc2, cam)
    np.testing.assert_array_equal(res["image"], res2["image"])
    np.testing.assert_array_equal(res["final_T"], res2["final_T"])


def test_transparent_scene_is_background():
    sc, cam = random_small(3, n=50)
    sc["opacity_logits"][:] = np.float32(-6.0)   # sigmoid < 1/255
    bg = (0.1, 0.2, 0.3)
    res = oracle.render(sc, cam, background=bg)
    np.testing.assert_array_equal(res["image"], np.broadcast_to(np.array(bg)[:, None, None], res["image"].shape))
    assert (res["final_T"] == 1).all() and (res["n_contrib"] == 0).all()


@pytest.mark.parametrize("seed", range(5))
def test_bruteforce_equals_tiled_when_alpha_below_bound(seed):
    """With every opacity below e^4.5/255 = 0.35301 no Gaussian can pass the
    1/255 test outside its 3-sigma square, so compositing every Gaussian at
    every pixel (no tiles) gives the tiled result."""
    sc, cam = random_small(seed, n=50, W=64, H=64, deg=2)
    sc["opacity_logits"] = np.minimum(sc["opacity_logits"], np.float32(-0.62))   # sigmoid(-0.62)=0.3498
    res = oracle.render(sc, cam)
    bf = oracle.bruteforce(res["proj"])
    np.testing.assert_allclose(res["image"], bf["image"], atol=1e-15)
    np.testing.assert_allclose(res["final_T"], bf["final_T"], atol=1e-15)


def test_bruteforce_differs_when_tiles_truncate():
    """Control for the test above: an opaque Gaussian whose 3-sigma square ends
    on a tile edge still reaches alpha > 1/255 one pixel further, in a tile it
    does not touch, so the brute force must disagree there."""
    cam = scenes.default_camera(64, 64)
    f = float(cam["fx"])
    sigma_w = 3 * math.sqrt(24.0 - 0.3) / f            # 2D variance 24 px^2 -> r = 15
    sc = tiny_scene([0, 0, 0], [math.log(sigma_w)] * 3, [1, 0, 0, 0], [8.0], rgb=[[1.0], [1.0], [1.0]])
    res = oracle.render(sc, cam)
    assert res["proj"]["radius"][0] == 15                # square covers pixels 17..47
    bf = oracle.bruteforce(res["proj"])
    assert (res["image"][:, 32, 48] == 0).all()
    assert bf["image"][0, 32, 48] > 1 / 255


# --------------------------------------------------------------------------- binning and sort

def _pixel_rect_tiles(u, v, r, W, H):
    """Tiles holding any pixel within Chebyshev distance r of (u, v), by
    visiting every pixel."""
    xs = np.arange(W)
    ys = np.arange(H)
    inx = np.abs(xs - u) <= r
    iny = np.abs(ys - v) <= r
    tiles = set()
    for y in ys[iny]:
        for x in xs[inx]:
            tiles.add((y // 16, x // 16))
    return tiles


@pytest.mark.parametrize("seed", range(3))
def test_binning_against_pixel_enumeration(seed):
    sc = scenes.make_scene("C1", n=300, seed=seed)
    sc["means"][0] *= np.float32(1.6)   # push some off screen
    cam = scenes.default_camera(100, 70)   # ragged tiles on both axes
    p = oracle.project(sc, cam)
    for i in range(p["n"]):
        if p["radius"][i] == 0 and p["tiles_touched"][i] == 0:
            g = oracle.debug_geometry(cam, sc["means"][:, i].astype(np.float64),
                                      sc["log_scales"][:, i].astype(np.float64),
                                      sc["quats"][:, i].astype(np.float64))
            if g is None:
                continue
            assert not _pixel_rect_tiles(g["u"], g["v"], g["radius"], 100, 70)
            continue
        ref = _pixel_rect_tiles(p["mean2d"][0, i], p["mean2d"][1, i], p["radius"][i], 100, 70)
        x0, y0, x1, y1 = p["rect"][:, i]
        got = {(ty, tx) for ty in range(y0, y1) for tx in range(x0, x1)}
        assert got == ref
        assert p["tiles_touched"][i] == len(ref)


def test_keys_sort_ranges_against_numpy():
    sc = scenes.make_scene("C1", n=400, seed=7)
    cam = scenes.default_camera(100, 70)
    p = oracle.project(sc, cam)
    offsets, keys, values = oracle.bin_pairs(p)
    tt = p["tiles_touched"].astype(np.uint64)
    np.testing.assert_array_equal(offsets, np.concatenate([[0], np.cumsum(tt)[:-1]]).astype(np.uint64))
    # emission order and key layout, rebuilt per Gaussian
    j = 0
    for i in range(p["n"]):
        x0, y0, x1, y1 = p["rect"][:, i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                assert keys[j] == ((ty * p["tiles_x"] + tx) << 32) | int(p["depth_bits"][i])
                assert values[j] == i
                j += 1
    assert j == len(keys)
    sk, sv = oracle.sort_pairs(keys, values)
    order = np.lexsort((values, keys))
    np.testing.assert_array_equal(sk, keys[order])
    np.testing.assert_array_equal(sv, values[order])
    T = p["tiles_x"] * p["tiles_y"]
    ranges = oracle.tile_ranges(sk, T)
    tiles = (sk >> np.uint64(32)).astype(np.int64)
    np.testing.assert_array_equal(ranges[:, 0], np.searchsorted(tiles, np.arange(T), "left"))
    np.testing.assert_array_equal(ranges[:, 1], np.searchsorted(tiles, np.arange(T), "right"))
    np.testing.assert_array_equal(oracle.tile_counts(p), np.bincount(tiles, minlength=T))
    for t in range(T):
        np.testing.assert_array_equal(oracle.tile_list(p, t), sv[ranges[t, 0]:ranges[t, 1]])


def test_depth_bits_are_float32_rounding():
    sc = scenes.make_scene("C1", n=500, seed=8)
    p = oracle.project(sc, scenes.default_camera(64, 64))
    vis = p["tiles_touched"] > 0
    np.testing.assert_array_equal(p["depth_bits"][vis], p["depth"][vis].astype(np.float32).view(np.uint32))
    # camera-space depth of the default camera is z + 3, exactly (float32 inputs)
    np.testing.assert_array_equal(p["depth"][vis], sc["means"][2][vis].astype(np.float64) + 3.0)


def test_culls():
    cam = scenes.default_camera(32, 32)
    mu = [[0, 0, 0, 0, 0], [0, 0, 0, 0, 0], [-2.9, -2.85, 0, 0, np.nan]]
    q = [[1, 1, 0, 1, 1], [0, 0, 0, 0, 0], [0, 0, 0, 0, 0], [0, 0, 0, 0, 0]]
    sc = tiny_scene(mu, np.full((3, 5), -3.0), q, np.zeros(5), rgb=np.full((3, 5), 0.5))
    p = oracle.project(sc, cam)
    # z_cam = 0.1 (behind near 0.2) culled; 0.15 culled; zero quaternion culled; NaN culled
    assert list(p["tiles_touched"] > 0) == [False, False, False, True, False]
    assert list(p["radius"] > 0) == [False, False, False, True, False]


def test_composite_pixels_and_tile_list_equal_the_whole_frame_path():
    """The per-tile entry points the full-size tests use (``tile_list`` and
    ``composite_pixels``) against the whole-frame path (emitted pairs sorted by
    qsort, ``composite`` over every pixel): same lists, and bit for bit the
    same colour, final T, n_contrib and decision margins on every pixel of
    every tile, the ragged right column and bottom row included."""
    sc = scenes.make_scene("C2", n=6000, seed=77)
    cam = scenes.look_at_camera([0.9, -0.6, -2.8], 203, 115)   # ragged: 13 x 8 tiles
    o = oracle.render(sc, cam, background=(0.1, 0.2, 0.3))
    proj = o["proj"]
    tx, ty = proj["tiles_x"], proj["tiles_y"]
    W, H = cam["width"], cam["height"]
    checked = 0
    for t in range(tx * ty):
        s, e = (int(v) for v in o["ranges"][t])
        lst = o["values"][s:e]
        np.testing.assert_array_equal(oracle.tile_list(proj, t), lst, err_msg=f"tile {t}")
        x0, y0 = (t % tx) * 16, (t // tx) * 16
        ys, xs = np.mgrid[y0:min(y0 + 16, H), x0:min(x0 + 16, W)]
        xs, ys = xs.ravel(), ys.ravel()
        o5, marg = oracle.composite_pixels(proj, xs, ys, lst, background=(0.1, 0.2, 0.3))
        np.testing.assert_array_equal(o5[:, :3], o["image"][:, ys, xs].T)
        np.testing.assert_array_equal(o5[:, 3], o["final_T"][ys, xs])
        np.testing.assert_array_equal(o5[:, 4], o["n_contrib"][ys, xs])
        np.testing.assert_array_equal(marg[:, 0], o["margin_alpha"][ys, xs])
        np.testing.assert_array_equal(marg[:, 1], o["margin_T"][ys, xs])
        checked += len(xs)
    assert checked == W * H
    assert len(o["keys"]) > 20 * tx * ty   # lists long enough to terminate pixels
    assert (o["n_contrib"] > 0).mean() > 0.5


def test_render_tiles_equals_the_whole_frame_path():
    """render_tiles (each tile's list from its row's candidates) against
    render (every pair emitted, qsort, composite): bit for bit on every pixel,
    for all tiles and for a scattered subset (other pixels untouched)."""
    sc = scenes.make_scene("C3", n=8000, seed=78)
    cam = scenes.look_at_camera([-0.8, 0.5, -2.9], 237, 141)   # ragged: 15 x 9 tiles
    o = oracle.render(sc, cam, background=(0.3, 0.1, 0.2))
    t = oracle.render_tiles(o["proj"], background=(0.3, 0.1, 0.2))
    for k in ("image", "final_T", "n_contrib", "margin_alpha", "margin_T"):
        np.testing.assert_array_equal(t[k], o[k], err_msg=k)
    T = o["proj"]["tiles_x"] * o["proj"]["tiles_y"]
    pick = np.random.default_rng(5).choice(T, 17, replace=False)
    sub = oracle.render_tiles(o["proj"], pick, background=(0.3, 0.1, 0.2))
    mask = np.zeros((141, 237), bool)
    for tile in pick:
        x0, y0 = (tile % o["proj"]["tiles_x"]) * 16, (tile // o["proj"]["tiles_x"]) * 16
        mask[y0:y0 + 16, x0:x0 + 16] = True
    np.testing.assert_array_equal(sub["image"][:, mask], o["image"][:, mask])
    np.testing.assert_array_equal(sub["n_contrib"][mask], o["n_contrib"][mask])
    assert not sub["image"][:, ~mask].any() and not sub["final_T"][~mask].any()
