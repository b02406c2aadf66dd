"""Host-only checks of the C ABI: the library loads, exports every function
include/gsmi.h declares, and rejects bad arguments before touching a device
(gs_validate never calls into HIP)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2607_15951_amd as gs
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "gsmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gs.LIB_PATH):
        pytest.fail("libgsmi.so is not built (python -m paper_2607_15951_amd.build)")
    return gs.load_library()


def test_header_declares_expected_entry_points():
    assert header_functions() == sorted(gs.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def _valid_args(n=10):
    g = gs.gs_gaussians()
    g.n = n
    g.sh_degree = 0
    g.attr_dtype = gs.GS_F32
    g.means = g.log_scales = g.quats = g.opacity_logits = g.sh = 0x1000   # never dereferenced
    cam = gs.make_camera(scenes.default_camera(64, 48))
    opts = gs.make_opts()
    return g, cam, opts


def test_validate_accepts_good_arguments(lib):
    g, cam, opts = _valid_args()
    assert gs.validate(g, cam, 64, 48, opts, C.c_void_p(0x2000)) == gs.GS_OK
    assert gs.validate(g, cam, 64, 48, None, C.c_void_p(0x2000)) == gs.GS_OK
    g.n = 0
    g.means = g.log_scales = g.quats = g.opacity_logits = g.sh = None
    assert gs.validate(g, cam, 1, 1, opts, C.c_void_p(0x2000)) == gs.GS_OK


def test_validate_bounds_the_pair_capacity(lib):
    """Pair offsets are 32-bit: a capacity above 2^32 - 1 is refused on the host."""
    g, cam, opts = _valid_args()
    opts.pair_capacity = (1 << 32) - 1
    assert gs.validate(g, cam, 64, 48, opts, C.c_void_p(0x2000)) == gs.GS_OK
    opts.pair_capacity = 1 << 32
    assert gs.validate(g, cam, 64, 48, opts, C.c_void_p(0x2000)) == gs.GS_ERR_UNSUPPORTED


def test_validate_accepts_the_reuse_flags(lib):
    g, cam, opts = _valid_args()
    for flags in (gs.RENDER_REUSE_ORDER, gs.RENDER_REUSE_LISTS, gs.RENDER_REUSE_ORDER | gs.RENDER_REUSE_LISTS):
        opts.flags = flags
        assert gs.validate(g, cam, 64, 48, opts, C.c_void_p(0x2000)) == gs.GS_OK, flags


@pytest.mark.parametrize("case", ["null_out", "neg_n", "huge_n", "deg4", "deg_neg", "dtype", "null_attr",
                                  "w0", "h0", "w_big", "nan_cam", "inf_t", "fx0", "near0", "tile8",
                                  "flags", "nan_bg"])
def test_validate_rejects(lib, case):
    g, cam, opts = _valid_args()
    out = C.c_void_p(0x2000)
    W, H = 64, 48
    if case == "null_out":
        out = None
    elif case == "neg_n":
        g.n = -1
    elif case == "huge_n":
        g.n = 1 << 31
    elif case == "deg4":
        g.sh_degree = 4
    elif case == "deg_neg":
        g.sh_degree = -1
    elif case == "dtype":
        g.attr_dtype = 7
    elif case == "null_attr":
        g.quats = None
    elif case == "w0":
        W = 0
    elif case == "h0":
        H = 0
    elif case == "w_big":
        W = 40000
    elif case == "nan_cam":
        cam.R[4] = float("nan")
    elif case == "inf_t":
        cam.t[2] = float("inf")
    elif case == "fx0":
        cam.fx = 0.0
    elif case == "near0":
        cam.near_plane = 0.0
    elif case == "tile8":
        opts.tile_size = 8
    elif case == "flags":
        opts.flags = 4          # only GS_RENDER_REUSE_ORDER (1) and GS_RENDER_REUSE_LISTS (2) are defined
    elif case == "nan_bg":
        opts.background[1] = float("nan")
    st = gs.validate(g, cam, W, H, opts, out)
    assert st == gs.GS_ERR_INVALID_ARGUMENT, (case, st)
    assert lib.gs_last_error(None).decode() != ""


def test_null_context_calls_fail_cleanly(lib):
    info = gs.gs_list_info()
    assert lib.gs_get_list_info(None, C.byref(info)) == gs.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_copy_projection(None, None, None, None, None, None, None) == gs.GS_ERR_INVALID_ARGUMENT
    lib.gs_destroy(None)


def test_bf16_storage_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(0, 3, 10000).astype(np.float32)
    ours = scenes.bf16_to_f32(scenes.to_bf16_storage(x))
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_binding_rejects_bad_tensors():
    """The binding checks device, dtype, contiguity and shape of every tensor
    before a pointer reaches the C ABI (which cannot see them)."""
    torch = pytest.importorskip("torch")
    import paper_2607_15951_amd as gs
    n = 10
    base = {"sh_degree": 1, "attr_dtype": gs.GS_F32,
            "means": torch.zeros((3, n)), "log_scales": torch.zeros((3, n)), "quats": torch.zeros((4, n)),
            "opacity_logits": torch.zeros(n), "sh": torch.zeros((4, 3, n))}
    with pytest.raises(ValueError, match="cuda"):
        gs.make_gaussians(base)                       # host tensors
    with pytest.raises(ValueError):
        gs.make_gaussians(dict(base, means=torch.zeros((2, n))))
    with pytest.raises(ValueError):
        gs.make_gaussians(dict(base, sh_degree=7))


def test_scene_from_rows_layout():
    """Rows [N, C] to the channel-major layout the C ABI takes (host tensors:
    the conversion is layout only), and its shape checks."""
    torch = pytest.importorskip("torch")
    import paper_2607_15951_amd as gs
    n, deg = 7, 2
    g = torch.Generator().manual_seed(3)
    means, ls, q = torch.randn(n, 3, generator=g), torch.randn(n, 3, generator=g), torch.randn(n, 4, generator=g)
    op, sh = torch.randn(n, generator=g), torch.randn(n, (deg + 1) ** 2, 3, generator=g)
    d = gs.scene_from_rows(means, ls, q, op, sh)
    assert d["sh_degree"] == deg and d["attr_dtype"] == gs.GS_F32
    assert d["means"].shape == (3, n) and torch.equal(d["means"][1], means[:, 1])
    assert d["quats"].shape == (4, n) and torch.equal(d["quats"][0], q[:, 0])
    assert d["sh"].shape == ((deg + 1) ** 2, 3, n) and torch.equal(d["sh"][4, 2], sh[:, 4, 2])
    assert all(d[k].is_contiguous() for k in ("means", "log_scales", "quats", "opacity_logits", "sh"))
    b = gs.scene_from_rows(means, ls, q, op, sh, gs.GS_BF16)
    assert b["sh"].dtype == torch.bfloat16 and b["means"].dtype == torch.float32
    with pytest.raises(ValueError):
        gs.scene_from_rows(means, ls, q, op, torch.randn(n, 5, 3))


def test_tune_candidates_match_the_header():
    """The binding's candidate list is the order of gs_autotune's out_ms
    array, whose length the header fixes."""
    text = open(os.path.join(ROOT, "include", "gsmi.h")).read()
    n = int(re.search(r"#define\s+GS_TUNE_CANDIDATES\s+(\d+)", text).group(1))
    assert len(gs.TUNE_CANDIDATES) == n
    listed = re.search(r"of every candidate in the order (.*?)\n \* Profiling", text, flags=re.S).group(1)
    values = [int(v) for v in re.findall(r"-?\d+", listed)]
    assert values == [v for _, v in gs.TUNE_CANDIDATES]
