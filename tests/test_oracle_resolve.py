"""Oracle pins for the ray-traced resolve (3.2.2) and the quantities it hands
to the reconstruction (3.2.3-3.2.4): the near weight across its ramp around
the focus plane, the per-field CoC means, the accumulated CoC c_t, and the
mip level eq. (8) takes from c_t.  Every expected value comes from the
thin-lens closed forms below (binary64), not from the oracle."""

import dataclasses
import math

import numpy as np
import pytest

from paper_2210_06158_amd import synth

SQRT2 = math.sqrt(2.0)


def coc_closed(lens, W, z):
    """Thin-lens CoC diameter in full-res pixels: a f |z - d| / (z (d - f))
    scaled by W / w_s (sections 1.1 and 3.3); its sqrt(2) level sets are the
    two bounds of eq. (6)."""
    a, f, d, ws = lens.focal / lens.fnum, lens.focal, lens.focus, lens.sensor
    return a * f * abs(z - d) / (z * (d - f)) * W / ws


def near_bound(lens, W):
    """Eq. (6)'s near bound of the zone of focus with w_i = W, solved for z."""
    a, f, d, ws = lens.focal / lens.fnum, lens.focal, lens.focus, lens.sensor
    return a * f * d * W / (a * f * W + SQRT2 * (d - f) * ws)


def near_weight(lens, W, z):
    """Near share of a hit at view depth z: 1/2 at the focus plane, rising
    linearly towards the camera and reaching 1 at the near bound z_nb
    (saturated beyond), i.e. a ramp of width 2 (d - z_nb) centred on d."""
    d, znb = lens.focus, near_bound(lens, W)
    return min(1.0, max(0.0, 0.5 + (d - z) / (2.0 * (d - znb))))


def plane(z, extent=400.0):
    return synth.quad((-extent, -extent, z), (-extent, extent, z), (extent, extent, z), (extent, -extent, z))


def flat_gbuffer(orc, W, H, z, colour=0.5):
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 2] = -1.0
    return orc.GBuffer(np.full((H, W, 4), colour, np.float32), np.full((H, W), z, np.float32), nrm)


LENS = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
W, H = 128, 96


def test_closed_forms_agree():
    """The near bound is where the CoC closed form equals sqrt(2), and the
    ramp reaches its ends there and at its mirror 2d - z_nb."""
    znb = near_bound(LENS, W)
    assert coc_closed(LENS, W, znb) == pytest.approx(SQRT2, rel=1e-12)
    assert near_weight(LENS, W, znb) == pytest.approx(1.0, abs=1e-12)
    assert near_weight(LENS, W, 2 * LENS.focus - znb) == pytest.approx(0.0, abs=1e-12)
    assert near_weight(LENS, W, LENS.focus) == 0.5


@pytest.mark.parametrize("z", [4.75, 5.2, 5.3])
def test_near_weight_and_field_coc_inside_the_ramp(orc, z):
    """One plane facing the camera at view depth z inside the ramp, every
    half-res pixel traced (mask mode all): every ray hits the plane at depth
    z, so each pixel's hit ratio is the near weight of z, N = n times it,
    both field colours are the plane's shading, both per-field CoC means are
    the closed-form CoC of z (a diameter in full-res pixels), and the mean far
    hit lies on the plane.  z sits where a half-width ramp (saturating at
    |z - d| = (d - z_nb) / 2) or a ramp centred on z_nb would give another
    weight, and where the CoC is far from its half (a radius)."""
    d, znb = LENS.focus, near_bound(LENS, W)
    w = near_weight(LENS, W, z)
    assert 0.05 < w < 0.95
    assert abs(z - d) > (d - znb) / 2                     # a half-width ramp would saturate
    w_nb_centred = min(1.0, max(0.0, 0.5 + (znb - z) / (2 * (d - znb))))
    assert abs(w_nb_centred - w) > 0.1
    sc = orc.OracleScene(synth.Scene(plane(z), np.array([[0.6, 0.5, 0.4]] * 2, np.float32),
                                     light_dir=synth.f32tuple(synth._normalize((0.2, -0.3, 1.0)))))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    m = 4
    o = orc.render_frame(sc, cam, LENS, synth.Params(mask_mode=synth.MASK_ALL, m=m), flat_gbuffer(orc, W, H, z))
    assert np.all(o["mask"] == m) and np.all(o["ray_hit"] >= 0)
    R0, R1, R2, R3 = o["resolve"]
    np.testing.assert_allclose(R1[..., 3], w, rtol=0, atol=2e-6)            # hit ratio
    np.testing.assert_allclose(R0[..., 3], m * w, rtol=0, atol=8e-6)        # N
    c = coc_closed(LENS, W, z)
    np.testing.assert_allclose(R2[..., 0], c, rtol=2e-5, atol=0)            # near-field CoC
    np.testing.assert_allclose(R2[..., 1], c, rtol=2e-5, atol=0)            # far-field CoC
    # Lambert: the normal facing the ray is -z, the light travels along L
    L = np.asarray(synth._normalize((0.2, -0.3, 1.0)))
    shade = np.array([0.6, 0.5, 0.4]) * (1.0 * L[2] + 0.15)
    np.testing.assert_allclose(R0[..., :3], np.broadcast_to(shade, R0[..., :3].shape), rtol=0, atol=2e-6)
    np.testing.assert_allclose(R1[..., :3], np.broadcast_to(shade, R1[..., :3].shape), rtol=0, atol=2e-6)
    np.testing.assert_allclose(R3[..., 2], z, rtol=2e-6, atol=0)            # mean far hit on the plane
    assert np.all(R3[..., 3] == 1.0)


@pytest.fixture(scope="module")
def bar_frame(orc):
    """A thin vertical bar at depth 2 (nearer than z_nb: fully near field) in
    front of a wall at depth 20 (beyond 2d - z_nb: fully far field), every
    half-res pixel traced with 64 rays, no history."""
    d, znb = LENS.focus, near_bound(LENS, W)
    zb, zw = 2.0, 20.0
    assert zb < znb and zw > 2 * d - znb
    bar = synth.quad((-0.01, -5, zb), (-0.01, 5, zb), (0.01, 5, zb), (0.01, -5, zb))
    scene = synth.Scene(np.concatenate([bar, plane(zw, 500.0)]),
                        np.array([[1.0, 0.2, 0.2]] * 2 + [[0.2, 0.3, 0.9]] * 2, np.float32))
    sc = orc.OracleScene(scene)
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    gb = orc.gbuffer(sc, cam, LENS)
    o = orc.render_frame(sc, cam, LENS, synth.Params(mask_mode=synth.MASK_ALL, m=64), gb)
    return dict(o=o, gb=gb, zb=zb, zw=zw)


def test_field_coc_comes_from_the_hits_not_the_gbuffer(bar_frame):
    """Pixels whose rays partly hit the bar: the near-field CoC mean is the
    CoC of the bar's depth and the far-field one that of the wall's, both
    closed forms, whatever the pixel's own G-buffer depth -- among them are
    pixels whose pinhole ray hits the bar, so a far-field CoC taken from the
    G-buffer would be the bar's.  The mean far hit lies on the wall."""
    o, gb, zb, zw = bar_frame["o"], bar_frame["gb"], bar_frame["zb"], bar_frame["zw"]
    R0, R1, R2, R3 = o["resolve"]
    h = R1[..., 3]
    mixed = (h > 0.02) & (h < 0.98)
    assert mixed.sum() >= 2 * (H // 2)
    cb, cw = coc_closed(LENS, W, zb), coc_closed(LENS, W, zw)
    assert cb > 20.0 and 10.0 < cw < 15.0
    np.testing.assert_allclose(R2[..., 0][mixed], cb, rtol=2e-5, atol=0)
    np.testing.assert_allclose(R2[..., 1][mixed], cw, rtol=2e-5, atol=0)
    np.testing.assert_allclose(R3[..., 2][mixed], zw, rtol=2e-6, atol=0)
    # the hit ratio is the share of rays on the bar: N / n with n = 64
    np.testing.assert_allclose(h, R0[..., 3] / 64.0, rtol=0, atol=1e-7)
    assert np.all(np.abs(h * 64.0 - np.round(h * 64.0)) < 1e-4)
    # some mixed pixels see the bar in the G-buffer (the half-res reduce takes
    # the nearest depth of each 2 x 2 quad)
    zq = gb.depth.reshape(H // 2, 2, W // 2, 2).min(axis=(1, 3))
    assert np.any(mixed & (zq == np.float32(zb)))
    # pixels away from the bar: every ray on the wall
    far = h == 0.0
    assert far.sum() > 0.5 * far.size
    np.testing.assert_allclose(R2[..., 1][far], cw, rtol=2e-5, atol=0)
    assert np.all(R2[..., 0][far] == 0.0)


def test_accumulated_coc_is_the_hit_ratio_blend(bar_frame):
    """Without history the accumulated CoC c_t (the reconstruction's kernel
    diameter, full-res pixels) is lerp(c_far, c_near, h) with this frame's
    hit ratio h (3.2.3), from the closed-form CoCs of the two depths."""
    o, zb, zw = bar_frame["o"], bar_frame["zb"], bar_frame["zw"]
    h = o["resolve"][1][..., 3].astype(np.float64)
    cb, cw = coc_closed(LENS, W, zb), coc_closed(LENS, W, zw)
    T1 = o["temporal"][1]
    np.testing.assert_allclose(T1[..., 0], cw + h * (cb - cw), rtol=2e-5, atol=0)
    np.testing.assert_allclose(T1[..., 1], h, rtol=0, atol=1e-7)


# ---------------------------------------------------------------- eq. (8)

def _box_mips(img, levels):
    """2 x 2 box mip chain (sizes halve exactly here)."""
    out = [img]
    for _ in range(levels):
        a = out[-1]
        out.append(0.25 * ((a[0::2, 0::2] + a[0::2, 1::2]) + (a[1::2, 0::2] + a[1::2, 1::2])))
    return out


def _bilinear(img, x, y):
    """Bilinear sample at texel coordinates (x, y), clamp to edge."""
    h, w = img.shape[:2]
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = x - x0, y - y0
    xa, xb = np.clip(x0, 0, w - 1).astype(int), np.clip(x0 + 1, 0, w - 1).astype(int)
    ya, yb = np.clip(y0, 0, h - 1).astype(int), np.clip(y0 + 1, 0, h - 1).astype(int)
    top = img[ya, xa] * (1 - fx)[..., None] + img[ya, xb] * fx[..., None]
    bot = img[yb, xa] * (1 - fx)[..., None] + img[yb, xb] * fx[..., None]
    return top * (1 - fy)[..., None] + bot * fy[..., None]


def _trilinear_recon(orc, med, ct, b, lod_of, p, inner):
    """Reconstruction of 3.2.4 with every pixel ray traced: kernel radius
    c_t / 4 on the 81-tap rings, a tap rejected when its own c_t / 4 is below
    its distance, each tap sampled trilinearly between mip levels floor(lod)
    and the next at lod = lod_of(c_t), the accepted taps averaged and blended
    into the median by b (eq. 5)."""
    hh, hw = ct.shape
    mips = _box_mips(med[..., :3].astype(np.float64), 3)
    ox, oy, frac = (np.asarray(a, np.float64) for a in orc.gather_rings(synth.Lens(), synth.Params()))
    ys, xs = np.mgrid[inner[0], inner[1]]
    R = np.minimum(ct[ys, xs] * 0.25, p.r_max)
    lod = np.clip(lod_of(ct[ys, xs]), 0.0, p.lod_max)
    L0 = np.minimum(np.floor(lod).astype(int), 3)
    L1 = np.minimum(L0 + 1, 3)
    fl = lod - L0
    acc = np.zeros(ys.shape + (3,))
    cnt = np.zeros(ys.shape)
    for k in range(81):
        sx, sy = xs + ox[k] * R, ys + oy[k] * R
        ix = np.clip(np.floor(sx + 0.5).astype(int), 0, hw - 1)
        iy = np.clip(np.floor(sy + 0.5).astype(int), 0, hh - 1)
        ok = ~(ct[iy, ix] * 0.25 < R * frac[k])
        s = np.zeros(ys.shape + (3,))
        for L in range(4):
            sc = 0.5 ** L
            v = _bilinear(mips[L], (sx + 0.5) * sc - 0.5, (sy + 0.5) * sc - 0.5)
            s += v * (((L0 == L) * (1 - fl)) + ((L1 == L) * fl))[..., None]
        acc += s * ok[..., None]
        cnt += ok
    nb = acc / cnt[..., None]
    m = med[ys, xs, :3].astype(np.float64)
    return m + (nb - m) * b[ys, xs][..., None]


def test_reconstruction_mip_level_follows_eq8_in_diameter_pixels(orc):
    """Eq. (8) with c_t a CoC diameter in full-res pixels: lod = c_t * 0.05.
    A colour field quadratic in x enters the ray-traced image through the
    history of a static near plane (as in the linear-field pin), so the mip
    levels differ from one another and the level blend shows in the result.
    The expected reconstruction is the plain numpy restatement above on the
    oracle's median input and c_t; the same restatement with lod taken from
    a radius (c_t / 4 * 0.05) misses the oracle by far more than the
    tolerance."""
    Wq, Hq, z = 128, 96, 2.0
    hw, hh = Wq // 2, Hq // 2
    np_ = hw * hh
    sc = orc.OracleScene(synth.Scene(plane(z), np.array([[0.6, 0.5, 0.4]] * 2, np.float32)))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, Wq, Hq)
    p = synth.Params(mask_mode=synth.MASK_ALL, m=4)
    gb = flat_gbuffer(orc, Wq, Hq, z)
    f0 = orc.render_frame(sc, cam, LENS, p, gb)
    hist = f0["hist_out"].copy()
    X = np.arange(hw, dtype=np.float32)
    A = hist[:4 * np_].reshape(hh, hw, 4)
    A[..., 0] = np.float32(0.1) + np.float32(0.0005) * X * X
    A[..., 1] = np.float32(1.5) - np.float32(0.0003) * X * X
    A[..., 2] = np.float32(0.3) + np.float32(0.02) * np.abs(X - np.float32(31.5))
    A[..., 3] = 1.0
    C = hist[8 * np_:12 * np_].reshape(hh, hw, 4)
    C[..., 2] = 0.0
    C[..., 3] = 1.0                                    # large variance: b at its cap
    f1 = orc.render_frame(sc, dataclasses.replace(cam, frame=1), LENS, p, gb, hist_in=hist, prev_cam=cam,
                          prev_lens=LENS)
    ct = f1["temporal"][1][..., 0].astype(np.float64)
    np.testing.assert_allclose(ct, coc_closed(LENS, Wq, z), rtol=2e-5)   # c_t: diameter in full-res px
    lod = ct * p.lod_scale
    assert 1.0 < lod.min() and lod.max() < 2.0        # levels 1 and 2 blended
    b = np.clip(f1["var_blur"].astype(np.float64) * p.var_recon_w, 0.0, p.b_max)
    assert b.min() > 0.5
    R = float(ct.max()) * 0.25
    mg = int(math.ceil(R)) + 9
    inner = (slice(mg, hh - mg), slice(mg, hw - mg))
    med = f1["rtmed"]
    want = _trilinear_recon(orc, med, ct, b, lambda c: c * p.lod_scale, p, inner)
    got = f1["recon"][inner][..., :3]
    np.testing.assert_allclose(got, want, rtol=0, atol=3e-5)
    wrong = _trilinear_recon(orc, med, ct, b, lambda c: c * 0.25 * p.lod_scale, p, inner)
    assert np.abs(wrong - got).max() > 30 * 3e-5
