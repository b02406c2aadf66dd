"""Pins of the oracle's float32 error model (the ambiguity margins).

The oracle (``composite_pixel`` in ``oracle/gs_oracle.c``) marks a pixel as
ambiguous when one of its threshold decisions -- the 1/255 alpha test of
Eq. 1's term or the 1e-4 early-termination test -- lies within a float32
error bound of the threshold.  It claims two bounds:

* alpha: a float32 evaluation of alpha = min(0.99, sigma * exp(power)) stays
  within e_a / 2 (relative) of the FP64 value, with
  e_a = 16 u (1 + (|A dx^2| + |C dy^2|) / 2 + |B dx dy|), u = 2^-24, and
  2u for an alpha clamped at 0.99;
* transmittance: after each composited entry T' = T (1 - a) stays within the
  accumulated relative bound e_T (each factor adds (e_a / 2) a / (1 - a) + u:
  the alpha bound, and one rounding of the update).

Here both are checked against an operation-by-operation float32 emulation of
the arithmetic a GPU evaluation performs: the projected centre stored as a
float hi/lo pair of the double value, re-expressed relative to the tile
origin in double and split again, the conic rounded to float32, the sigmoid
evaluated in double and rounded once,
the conic pre-scaled by -log2(e)/2, the quadratic form by two fused
multiply-adds, exp2, and T' = fma(-a, T, T).  Every float32 operation is
rounded to nearest (numpy's float32 arithmetic; fused multiply-adds with a
single rounding); the hardware exp2 is taken within 1 ulp of the exact value
(its published accuracy), by trying the correctly rounded value and both
neighbours.  A second check guards against an inflated bound: the worst error
seen must use a fair share of it.
"""
import math

import numpy as np

U = 2.0 ** -24
F = np.float32
LOG2E_F = F(1.4426950408889634)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def fma32(a, b, c):
    """float32 a * b + c with one rounding (a, b, c float32 arrays)."""
    p = a.astype(np.float64) * b.astype(np.float64)      # exact: 48-bit product
    c64 = c.astype(np.float64)
    s = p + c64
    bb = s - p                                           # TwoSum: s + t == p + c exactly
    t = (p - (s - bb)) + (c64 - bb)
    r = s.astype(np.float32)
    # s rounds correctly to float32 unless it sits exactly on a midpoint of two
    # float32 values, where the sign of t decides
    up = np.nextafter(r, np.float32(np.inf))
    dn = np.nextafter(r, np.float32(-np.inf))
    mid_up = (r.astype(np.float64) + up.astype(np.float64)) / 2
    mid_dn = (r.astype(np.float64) + dn.astype(np.float64)) / 2
    r = np.where((s == mid_up) & (t > 0), up, r)
    r = np.where((s == mid_dn) & (t < 0), dn, r)
    return r


def exp2_choices(x):
    """The float32 values a 1-ulp exp2 may return: RN(2^x) and its neighbours."""
    e = f32(np.exp2(x.astype(np.float64)))
    return (e, np.nextafter(e, np.float32(np.inf)), np.nextafter(e, np.float32(0)))


def draw_entries(rng, m):
    """m seeded (Gaussian, pixel) pairs: 2D covariances with eigenvalues in
    [0.3, 4000] px^2 (the EWA dilation is 0.3), centres up to 4 standard
    deviations from a pixel of a tile anywhere on a 4K screen, opacity
    logits N(0, 2)."""
    lam1 = np.exp(rng.uniform(math.log(0.3), math.log(4000.0), m))
    lam2 = np.exp(rng.uniform(math.log(0.3), math.log(4000.0), m))
    th = rng.uniform(0, math.pi, m)
    c, s = np.cos(th), np.sin(th)
    s11 = c * c * lam1 + s * s * lam2
    s22 = s * s * lam1 + c * c * lam2
    s12 = c * s * (lam1 - lam2)
    det = s11 * s22 - s12 * s12
    A, B, C = s22 / det, -s12 / det, s11 / det
    ox = 16.0 * rng.integers(0, 240, m)
    oy = 16.0 * rng.integers(0, 135, m)
    lx = rng.integers(0, 16, m).astype(np.float64)
    ly = rng.integers(0, 16, m).astype(np.float64)
    # offset from the pixel at Mahalanobis distance d: (dx, dy) = L (cos phi, sin phi) d
    d = np.sqrt(rng.uniform(0.0, 16.0, m))
    phi = rng.uniform(0, 2 * math.pi, m)
    l11 = np.sqrt(s11)
    l21 = s12 / l11
    l22 = np.sqrt(s22 - l21 * l21)
    zx, zy = np.cos(phi) * d, np.sin(phi) * d
    u = (ox + lx) + l11 * zx
    v = (oy + ly) + l21 * zx + l22 * zy
    logit = f32(rng.normal(0.0, 2.0, m))
    return dict(A=A, B=B, C=C, u=u, v=v, ox=ox, oy=oy, lx=lx, ly=ly, logit=logit)


def oracle_alpha(e):
    """alpha and e_a exactly as the oracle computes them (double precision)."""
    op = 1.0 / (1.0 + np.exp(-e["logit"].astype(np.float64)))
    dx = e["u"] - (e["ox"] + e["lx"])
    dy = e["v"] - (e["oy"] + e["ly"])
    qa = e["A"] * dx * dx
    qc = e["C"] * dy * dy
    qb = e["B"] * dx * dy
    power = -0.5 * (qa + qc) - qb
    a = op * np.exp(power)
    ea = 16.0 * U * (1.0 + 0.5 * (np.abs(qa) + np.abs(qc)) + np.abs(qb))
    clamped = a > 0.99
    ea = np.where(clamped & (a > 0.99 * (1.0 + ea)), 2.0 * U, ea)
    a = np.where(clamped, 0.99, a)
    return a, ea


def gpu_alpha_candidates(e):
    """Every float32 alpha a GPU evaluation of the entry may produce (one per
    choice of the exp2 result)."""
    # the projection's outputs: centre as hi/lo float pair, conic and opacity
    uh, vh = f32(e["u"]), f32(e["v"])
    ul, vl = f32(e["u"] - uh.astype(np.float64)), f32(e["v"] - vh.astype(np.float64))
    A32, B32, C32 = f32(e["A"]), f32(e["B"]), f32(e["C"])
    # the sigmoid in double, rounded once to float32
    op32 = f32(1.0 / (1.0 + np.exp(-e["logit"].astype(np.float64))))
    # staging: centre relative to the tile origin in double, split again
    du = (uh.astype(np.float64) + ul.astype(np.float64)) - e["ox"]
    dv = (vh.astype(np.float64) + vl.astype(np.float64)) - e["oy"]
    du_hi, dv_hi = f32(du), f32(dv)
    du_lo, dv_lo = f32(du - du_hi.astype(np.float64)), f32(dv - dv_hi.astype(np.float64))
    c_half = F(-0.5) * LOG2E_F
    Ap = (c_half * A32).astype(np.float32)
    Bp = (-LOG2E_F * B32).astype(np.float32)
    Cp = (c_half * C32).astype(np.float32)
    # per pixel
    dx = ((du_hi - f32(e["lx"])) + du_lo).astype(np.float32)
    dy = ((dv_hi - f32(e["ly"])) + dv_lo).astype(np.float32)
    pw = fma32(fma32(Ap, dx, (Bp * dy).astype(np.float32)), dx, ((Cp * dy) * dy).astype(np.float32))
    return [np.minimum(F(0.99), (op32 * E).astype(np.float32)) for E in exp2_choices(pw)]


def test_alpha_within_half_the_oracle_bound():
    rng = np.random.default_rng(20260)
    worst = 0.0
    n_total = 0
    for _ in range(4):
        e = draw_entries(rng, 250_000)
        a64, ea = oracle_alpha(e)
        keep = a64 > 0            # below double range nothing is compared
        for a32 in gpu_alpha_candidates(e):
            rel = np.abs(a32.astype(np.float64) - a64)[keep] / (0.5 * ea[keep] * a64[keep])
            worst = max(worst, float(rel.max()))
        n_total += int(keep.sum())
    print(f"alpha: worst error = {worst:.3f} of e_a/2 over {n_total} entries")
    assert n_total >= 900_000
    assert worst <= 1.0, f"float32 alpha leaves the oracle's bound: {worst:.3f} x e_a/2"
    # the bound is not inflated: the worst case uses a fair share of it
    assert worst >= 0.05, f"bound is loose by {1 / worst:.0f}x"


def test_alpha_bound_near_the_threshold():
    """The decisions that matter: entries whose alpha lies within 1% of 1/255
    (the skip test) and within 1% of the 0.99 clamp (drawn with opaque logits
    near the centre)."""
    rng = np.random.default_rng(20261)
    e_skip = draw_entries(rng, 400_000)
    e_clamp = draw_entries(rng, 400_000)
    e_clamp["logit"] = f32(rng.normal(7.0, 2.0, 400_000))
    for e, lo, hi in ((e_skip, 0.99 / 255, 1.01 / 255), (e_clamp, 0.98, 1.0)):
        a64, ea = oracle_alpha(e)
        sel = (a64 >= lo) & (a64 <= hi)
        assert sel.sum() > 200, (lo, hi, int(sel.sum()))
        for a32 in gpu_alpha_candidates(e):
            err = np.abs(a32.astype(np.float64) - a64)[sel]
            assert (err <= 0.5 * ea[sel] * a64[sel]).all()
        # where the margin says unambiguous (>= 1), float32 takes the oracle's branch
        if lo < 0.01:
            margin = np.abs(255.0 * a64 - 1.0) / ea
            sure = sel & (margin >= 1.0)
            for a32 in gpu_alpha_candidates(e):
                assert ((a32[sure] >= F(1.0 / 255.0)) == (a64[sure] >= 1.0 / 255.0)).all()


def test_transmittance_bound_over_long_walks():
    """Walks of up to 1200 entries of small alphas: while both sides take the
    same decisions, the float32 T (one fused multiply-add per entry) stays
    within the oracle's accumulated bound e_T; where they part, the oracle's
    margin for that decision is below 1 (the pixel is marked ambiguous)."""
    rng = np.random.default_rng(20262)
    walks, length = 3000, 1200
    e = draw_entries(rng, walks * length)
    # mostly faint entries, so walks run long before terminating
    e["logit"] = f32(rng.normal(-4.0, 1.0, walks * length))
    a64, ea = oracle_alpha(e)
    a32s = gpu_alpha_candidates(e)
    a64 = a64.reshape(walks, length)
    ea = ea.reshape(walks, length)
    worst = 0.0
    composited = 0
    parted = 0
    for a32 in a32s:   # exp2 result RN, one ulp high, one ulp low
        a32 = a32.reshape(walks, length)
        T64 = np.ones(walks)
        eT = np.zeros(walks)
        T32 = np.ones(walks, np.float32)
        live = np.ones(walks, bool)
        m_alpha = np.full(walks, np.inf)
        m_T = np.full(walks, np.inf)
        for j in range(length):
            a, e_a, b = a64[:, j], ea[:, j], a32[:, j]
            m_alpha = np.minimum(m_alpha, np.where(live, np.abs(255.0 * a - 1.0) / e_a, np.inf))
            pass64 = a >= 1.0 / 255.0
            pass32 = b >= F(1.0 / 255.0)
            Tn = T64 * (1.0 - a)
            eTn = eT + 0.5 * e_a * a / (1.0 - a) + U
            Tn32 = fma32(-b, T32, T32)
            m_T = np.minimum(m_T, np.where(live & pass64, np.abs(Tn * 1e4 - 1.0) / eTn, np.inf))
            stop64 = pass64 & (Tn < 1e-4)
            stop32 = pass32 & (Tn32 < F(1e-4))
            differ = live & ((pass64 != pass32) | (stop64 != stop32))
            if differ.any():
                # the oracle flags every pixel whose decisions part
                assert (np.minimum(m_alpha, m_T)[differ] < 1.0).all()
                parted += int(differ.sum())
                live &= ~differ
            take = live & pass64 & ~stop64
            rel = np.abs(Tn32.astype(np.float64) - Tn) / Tn
            chk = take
            if chk.any():
                r = rel[chk] / eTn[chk]
                worst = max(worst, float(r.max()))
                assert (r <= 1.0).all(), f"T leaves the bound at step {j}: {float(r.max()):.3f}"
            composited += int(take.sum())
            T64 = np.where(take, Tn, T64)
            eT = np.where(take, eTn, eT)
            T32 = np.where(take, Tn32, T32)
            live &= ~stop64
    print(f"T: worst error = {worst:.3f} of e_T over {composited} composited steps; {parted} walks parted")
    assert composited > 500_000
    assert worst >= 0.02, f"T bound is loose by {1 / worst:.0f}x"


def emulate_tile_walk(rng, proj, list_idx, px, py, ox, oy):
    """float32 per-pixel walk of a GPU blend over one list, for pixels
    (px, py) of the tile with origin (ox, oy): alpha as above (each exp2
    result drawn at random within 1 ulp), T' = fma(-a, T, T), colour
    accumulated as fma(a T, rgb, C), the 1/255 skip and the 1e-4 stop."""
    n = proj["n"]
    k = len(px)
    Tr = np.ones(k, np.float32)
    col = np.zeros((3, k), np.float32)
    last = np.zeros(k, np.int64)
    done = np.zeros(k, bool)
    lx, ly = f32(px - ox), f32(py - oy)
    for j, i in enumerate(list_idx):
        e = dict(A=np.full(k, proj["conic"][0, i]), B=np.full(k, proj["conic"][1, i]),
                 C=np.full(k, proj["conic"][2, i]), u=np.full(k, proj["mean2d"][0, i]),
                 v=np.full(k, proj["mean2d"][1, i]), ox=np.full(k, float(ox)), oy=np.full(k, float(oy)),
                 lx=lx.astype(np.float64), ly=ly.astype(np.float64), logit=np.full(k, proj["logit"][i]))
        cands = gpu_alpha_candidates(e)
        pick = rng.integers(0, 3, k)
        al = np.choose(pick, cands)
        tn = fma32(-al, Tr, Tr)
        ok = al >= F(1.0 / 255.0)
        stop = ok & (tn < F(1e-4)) & ~done
        take = ok & ~stop & ~done
        done |= stop
        w = np.where(take, (al * Tr).astype(np.float32), F(0.0))
        for ch in range(3):
            col[ch] = fma32(w, np.full(k, f32(proj["rgb"][ch, i])), col[ch])
        Tr = np.where(take, tn, Tr)
        last = np.where(take, j + 1, last)
        if done.all():
            break
    return col, Tr, last


def test_ambiguous_mask_covers_every_float32_disagreement():
    """The property the image parity relies on: wherever the oracle marks a
    pixel unambiguous (both margins >= 1), a float32 walk of the same list
    yields the same n_contrib and an image and final T within 1e-4 of the
    oracle's.  Lists of 60 to 900 Gaussians around a tile, seeded; the
    oracle's margins come from ``composite_pixels`` itself."""
    import oracle
    rng = np.random.default_rng(20263)
    n_px = n_amb = 0
    worst = 0.0
    for trial in range(32):
        L = int(rng.integers(60, 900))
        ox, oy = 16 * int(rng.integers(0, 240)), 16 * int(rng.integers(0, 135))
        # Gaussians centred within 12 px of the tile, covariances as above
        e = draw_entries(rng, L)
        u = ox + rng.uniform(-12.0, 28.0, L)
        v = oy + rng.uniform(-12.0, 28.0, L)
        # from opaque to faint lists (long walks before termination)
        logit = f32(rng.normal((0.5, -1.5, -3.5, -5.0)[trial % 4], 1.0, L))
        proj = dict(n=L, mean2d=np.stack([u, v]), conic=np.stack([e["A"], e["B"], e["C"]]),
                    opacity=1.0 / (1.0 + np.exp(-logit.astype(np.float64))), logit=logit,
                    rgb=rng.uniform(0.0, 1.0, (3, L)))
        order = np.arange(L, dtype=np.uint32)
        ys, xs = np.mgrid[oy:oy + 16, ox:ox + 16]
        px, py = xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)
        o5, marg = oracle.composite_pixels(proj, px, py, order)
        col, Tr, last = emulate_tile_walk(rng, proj, order, px, py, ox, oy)
        amb = (marg[:, 0] < oracle.ALPHA_MARGIN) | (marg[:, 1] < oracle.T_MARGIN)
        good = ~amb
        d = np.abs(col.T.astype(np.float64) - o5[:, :3]).max(axis=1)
        dT = np.abs(Tr.astype(np.float64) - o5[:, 3])
        assert (last[good] == o5[good, 4]).all(), f"trial {trial}: n_contrib differs on an unambiguous pixel"
        assert d[good].max() <= 1e-4 and dT[good].max() <= 1e-4, f"trial {trial}"
        worst = max(worst, float(d[good].max()))
        n_px += len(px)
        n_amb += int(amb.sum())
    print(f"walks: {n_px} pixels, {n_amb} ambiguous, worst unambiguous max-abs {worst:.2e}")
    assert n_amb < 0.05 * n_px
