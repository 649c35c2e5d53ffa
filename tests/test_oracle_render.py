"""Oracle pins for the per-frame pass: mask (3.2.1, eqs. 2-4), post-process
filters (3.1), resolve and temporal accumulation (3.2.2-3.2.3), reconstruction
(3.2.4, eq. 5) and composite (3.3)."""

import dataclasses
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from paper_2210_06158_amd import synth


def plane_scene(z0, albedo=(0.6, 0.5, 0.4), extent=400.0):
    v = synth.quad((-extent, -extent, z0), (-extent, extent, z0), (extent, extent, z0), (extent, -extent, z0))
    return synth.Scene(v, np.array([albedo, albedo], np.float32),
                       light_dir=synth.f32tuple(synth._normalize((0.2, -0.3, 1.0))))


def gb_from_half(orc, depth_half, normal=(0.0, 0.0, -1.0), colour=(0.5, 0.5, 0.5)):
    hh, hw = depth_half.shape
    d = np.repeat(np.repeat(depth_half.astype(np.float32), 2, 0), 2, 1)
    H, W = d.shape
    n = np.zeros((H, W, 4), np.float32)
    n[..., :3] = normal
    c = np.ones((H, W, 4), np.float32)
    c[..., :3] = colour
    return orc.GBuffer(c, d, n)


@pytest.fixture(scope="module")
def small(orc):
    scene, cam, lens, params = synth.scene_small()
    sc = orc.OracleScene(scene)
    sc.build_bvh()
    gb = orc.gbuffer(sc, cam, lens)
    out = orc.render_frame(sc, cam, lens, params, gb)
    return dict(scene=scene, sc=sc, cam=cam, lens=lens, params=params, gb=gb, out=out)


# ---------------------------------------------------------------- composite

def test_pinhole_reduction_is_the_gbuffer(orc, small):
    """a = 0 (N = infinity): every CoC is 0, so every pixel is in the zone of
    focus and the output equals the sharp raster colour bit for bit."""
    lens = dataclasses.replace(small["lens"], fnum=math.inf)
    gb = orc.gbuffer(small["sc"], small["cam"], lens)
    out = orc.render_frame(small["sc"], small["cam"], lens, small["params"], gb)
    assert np.array_equal(out["colour"][..., :3].view(np.uint32), gb.colour[..., :3].view(np.uint32))


def test_in_focus_pixels_copy_raster_colour(orc, small):
    out, gb, lens = small["out"], small["gb"], small["lens"]
    H, W = gb.depth.shape
    valid = out["temporal"][0][..., 3] > 0
    hv = np.pad(valid, 1, mode="edge")
    # a full-res pixel blends the 4 half-res texels around (x/2 - 1/4, y/2 - 1/4)
    yy, xx = np.mgrid[0:H, 0:W]
    y0, x0 = (yy + 1) // 2 - 1, (xx + 1) // 2 - 1
    any_valid = np.zeros((H, W), bool)
    for dy in (0, 1):
        for dx in (0, 1):
            any_valid |= hv[np.clip(y0 + dy, 0, H // 2 - 1) + 1, np.clip(x0 + dx, 0, W // 2 - 1) + 1]
    coc = np.array([[orc.coc(lens, W, float(z)) for z in row] for row in gb.depth[:, ::1]])
    sel = (coc <= math.sqrt(2.0)) & ~any_valid
    assert sel.sum() > 1000
    assert np.array_equal(out["colour"][sel][:, :3].view(np.uint32), gb.colour[sel][:, :3].view(np.uint32))


# ---------------------------------------------------------------- ray mask

@pytest.mark.parametrize("z0,expect", [(40.0, 0), (15.0, 0), (3.0, 1)])
def test_mask_flat_plane(orc, z0, expect):
    """Constant depth and normal: no gradient, so x_n = 0; only an
    out-of-focus near-field pixel gets its single ray (3.2.1)."""
    lens = synth.Lens()
    sc = orc.OracleScene(plane_scene(z0))
    cam = synth.look_camera((0, 0, 0), 0, 0, 256, 64)
    gb = gb_from_half(orc, np.full((32, 128), z0))
    out = orc.render_frame(sc, cam, lens, synth.Params(m=6), gb)
    assert (out["mask"] == expect).all()


@pytest.mark.parametrize("alpha,count", [(0.25, 2), (1.0, 5), (4.0, 9)])
def test_mask_depth_ramp(orc, alpha, count):
    """d/z rising by alpha per half-res pixel: the unit-gain Sobel gives
    delta_d = alpha, so x = 0.8 alpha, x_n = 1 - 1/(x + 1) (eqs. 2, 3) and the
    ray count is round(x_n * m) (eq. 4 with zero variance)."""
    lens = synth.Lens(fnum=64.0)
    d = lens.focus
    qx = np.arange(128, dtype=np.float64)
    depth = np.tile(d / (alpha * qx + 1.0), (32, 1))
    sc = orc.OracleScene(plane_scene(20.0))
    cam = synth.look_camera((0, 0, 0), 0, 0, 256, 64)
    out = orc.render_frame(sc, cam, lens, synth.Params(m=12), gb_from_half(orc, depth))
    x = 0.8 * alpha
    want = math.floor((1.0 - 1.0 / (x + 1.0)) * 12 + 0.5)
    assert want == count
    assert (out["mask"][:, 4:124] == count).all()


@pytest.mark.parametrize("var,m,count", [(2e-6, 10, 2), (5e-6, 10, 5), (1e-5, 10, 10), (1e-3, 7, 7)])
def test_mask_variance_term(orc, var, m, count):
    """Eq. (4): x_f = saturate(x_n + var * 1e5) * m with the previous frame's
    blurred variance at the reprojected texel (static camera)."""
    lens = synth.Lens()
    sc = orc.OracleScene(plane_scene(40.0))
    cam = synth.look_camera((0, 0, 0), 0, 0, 128, 64)
    gb = gb_from_half(orc, np.full((32, 64), 40.0))
    npx = 32 * 64
    hist = orc.history_zeros(128, 64)
    hist[4 * npx + 3:8 * npx:4] = 1.0            # age
    hist[12 * npx:] = var                         # blurred variance
    out = orc.render_frame(sc, cam, lens, synth.Params(m=m), gb, hist_in=hist, prev_cam=cam, prev_lens=lens)
    assert (out["prev_idx"].ravel() == np.arange(npx)).all()
    assert (out["mask"] == count).all()


# ---------------------------------------------------------------- post-process

def test_tile_max_and_dilation(small):
    out, p = small["out"], small["params"]
    r = np.abs(out["colr"][..., 3])
    T = p.tile
    th, tw = out["tile_max"].shape
    pad = np.zeros((th * T, tw * T), np.float32)
    pad[:r.shape[0], :r.shape[1]] = r
    tmax = pad.reshape(th, T, tw, T).max(axis=(1, 3))
    assert np.array_equal(out["tile_max"], tmax)
    D = math.ceil(p.r_max / T)
    dil = ndi.maximum_filter(tmax, size=2 * D + 1, mode="constant", cval=0.0)
    assert np.array_equal(out["tile_dil"], dil)


def test_half_res_reduce(orc, small):
    out, gb, lens = small["out"], small["gb"], small["lens"]
    z = gb.depth
    quads = np.stack([z[0::2, 0::2], z[0::2, 1::2], z[1::2, 0::2], z[1::2, 1::2]])
    assert np.array_equal(out["zn"][..., 0], quads.min(0))
    r = out["colr"][..., 3]
    coc = np.array([[orc.coc(lens, 256, float(v)) for v in row] for row in quads.min(0)])
    np.testing.assert_allclose(np.abs(r), np.minimum(coc / 4, 32.0), rtol=1e-6)
    assert ((r < 0) == (quads.min(0) < lens.focus)).all() | (r == 0).all()


def test_median_postfilter_is_median(small):
    g = small["out"]["gather"][..., :3]
    pad = np.pad(g, ((1, 1), (1, 1), (0, 0)), mode="edge")
    stack = np.stack([pad[dy:dy + g.shape[0], dx:dx + g.shape[1]] for dy in range(3) for dx in range(3)])
    assert np.array_equal(small["out"]["ppmed"][..., :3], np.median(stack, axis=0).astype(np.float32))


@pytest.mark.parametrize("blades,polygon", [(0, 0), (6, 1), (5, 1)])
def test_constant_image_is_preserved(orc, blades, polygon):
    """Normalised filters leave a constant image constant (3.1.1-3.1.3),
    with the circular gather kernel and with the polygonal one."""
    lens = synth.Lens(blades=blades, blade_rot=0.4)
    sc = orc.OracleScene(plane_scene(3.0))
    cam = synth.look_camera((0, 0, 0), 0, 0, 128, 64)
    col = (0.3, 0.6, 0.9)
    out = orc.render_frame(sc, cam, lens, synth.Params(pp_polygon=polygon),
                           gb_from_half(orc, np.full((32, 64), 3.0), colour=col))
    for k in ("pre", "gather", "ppmed"):
        np.testing.assert_allclose(out[k][..., :3], np.broadcast_to(col, out[k][..., :3].shape), rtol=2e-5)


def _aperture_norm(x, y, lens):
    """Norm of the lens aperture (blade normals at rot + pi/B + 2 pi i/B,
    apothem cos(pi/B)) of the lens points behind gather offsets (x, y):
    the offsets are the aperture's far-field image reflected, (-px, py)."""
    B, rot = lens.blades, lens.blade_rot
    th = rot + math.pi / B + 2.0 * math.pi * np.arange(B) / B
    px, py = -np.asarray(x, np.float64), np.asarray(y, np.float64)
    return np.max(np.outer(px, np.cos(th)) + np.outer(py, np.sin(th)), axis=1) / math.cos(math.pi / B)


@pytest.mark.parametrize("blades,rot", [(6, 0.3), (5, 0.0), (8, 1.1)])
def test_polygon_gather_taps_lie_on_the_aperture(orc, blades, rot):
    """Section 2: polygonal bokeh by changing the shape of the sampling
    kernel.  Ring k's 8k taps lie on the aperture polygon scaled to k/4 (its
    own norm), one tap every 1/(8k) of the perimeter (chords between
    neighbours equal the step unless a corner lies between them)."""
    lens = synth.Lens(blades=blades, blade_rot=rot)
    ox, oy, fr = orc.gather_rings(lens, synth.Params(pp_polygon=1))
    assert ox[0] == 0.0 and oy[0] == 0.0 and fr[0] == 0.0
    side = 2.0 * math.sin(math.pi / blades)
    i = 1
    for k in range(1, 5):
        n = 8 * k
        sl = slice(i, i + n)
        assert np.all(fr[sl] == np.float32(0.25 * k))
        np.testing.assert_allclose(_aperture_norm(ox[sl], oy[sl], lens), k / 4.0, rtol=2e-6)
        step = (k / 4.0) * blades * side / n
        x, y = ox[sl].astype(np.float64), oy[sl].astype(np.float64)
        chords = np.hypot(np.diff(np.append(x, x[0])), np.diff(np.append(y, y[0])))
        assert np.all(chords <= step * (1 + 1e-5))
        if n > blades:      # some neighbours share an edge
            assert chords.max() == pytest.approx(step, rel=1e-5)
        i += n
    # without the flag (or without blades) the kernel stays circular
    for lz, pz in ((lens, synth.Params(pp_polygon=0)), (synth.Lens(blades=0), synth.Params(pp_polygon=1))):
        cx, cy, cf = orc.gather_rings(lz, pz)
        np.testing.assert_allclose(np.hypot(cx, cy), cf, atol=1e-6)


def test_all_in_focus_gather_is_identity(orc):
    lens = synth.Lens(fnum=math.inf)
    scene, cam, _, params = synth.scene_small()
    sc = orc.OracleScene(scene)
    gb = orc.gbuffer(sc, cam, lens)
    out = orc.render_frame(sc, cam, lens, params, gb)
    assert np.array_equal(out["gather"][..., :3], out["pre"][..., :3])


# ---------------------------------------------------------------- rays

def test_compaction_order(small):
    out = small["out"]
    m = out["mask"].ravel().astype(np.int64)
    q = np.flatnonzero(m)
    assert np.array_equal(out["queue"], q)
    base = np.concatenate([[0], np.cumsum(m[q])[:-1]])
    assert np.array_equal(out["ray_base"], base)
    assert out["n_rays"] == m.sum()


def test_thin_lens_at_zero_aperture_is_pinhole(orc):
    """a = 0: every lens point is the lens centre, so the ray towards the focus
    point is the pinhole ray; its hits match a half-resolution pinhole
    G-buffer away from depth discontinuities."""
    scene, cam, _, params = synth.scene_small()
    lens = synth.Lens(fnum=math.inf)
    sc = orc.OracleScene(scene)
    gb = orc.gbuffer(sc, cam, lens)
    out = orc.render_frame(sc, cam, lens, dataclasses.replace(params, mask_mode=synth.MASK_ALL, m=1), gb)
    half = dataclasses.replace(cam, width=128, height=128)
    ghalf = orc.gbuffer(sc, half, lens)
    z_ray = out["ray_col"][:, 3].reshape(128, 128)
    same = np.isclose(z_ray, ghalf.depth, rtol=1e-5) | (np.isinf(z_ray) & np.isinf(ghalf.depth))
    assert same.mean() > 0.995


def test_resolve_lerp_equals_sample_mean(small):
    """With both fields populated, lerp(far, near, h) is the plain mean of the
    pixel's ray colours (3.2.2)."""
    out = small["out"]
    R0, R1, R2 = (out["resolve"][i].reshape(-1, 4) for i in range(3))
    checked = 0
    for j, q in enumerate(out["queue"]):
        n = int(R2[q, 2])
        N = R0[q, 3]
        if not (0 < N < n):
            continue
        b = out["ray_base"][j]
        mean = out["ray_col"][b:b + n, :3].astype(np.float64).mean(0)
        h = R1[q, 3]
        lerp = R1[q, :3] + (R0[q, :3] - R1[q, :3]) * h
        np.testing.assert_allclose(lerp, mean, atol=2e-6)
        checked += 1
    assert checked > 50


def test_half_plane_occluder_hit_ratio(orc):
    """Near-field half-plane x < 0 at depth z1 in front of a far wall: the
    rays of a pixel cross depth z1 inside a disc of radius rho = (a/2)(d -
    z1)/d around the pixel's line of sight, so the hit ratio is the
    circular-segment fraction F(s) = (arccos s - s sqrt(1 - s^2)) / pi of that
    disc lying beyond the edge, s = signed distance / rho (3.2.2)."""
    lens = synth.Lens(fnum=1.4, focus=15.0)
    z1 = 0.5
    occ = synth.quad((-50, -50, z1), (-50, 50, z1), (0, 50, z1), (0, -50, z1))
    wall = synth.quad((-500, -500, 60), (-500, 500, 60), (500, 500, 60), (500, -500, 60))
    scene = synth.Scene(np.concatenate([occ, wall]), np.ones((4, 3), np.float32))
    sc = orc.OracleScene(scene)
    cam = synth.look_camera((0, 0, 0), 0, 0, 1024, 8)
    gb = orc.gbuffer(sc, cam, lens)
    out = orc.render_frame(sc, cam, lens, synth.Params(m=255, mask_mode=synth.MASK_ALL), gb)
    h = out["resolve"][1][..., 3]                                   # hit ratio per pixel
    a = lens.focal / lens.fnum
    rho = 0.5 * a * (lens.focus - z1) / lens.focus
    tx = synth.half_fov_tan(lens)
    qx = np.arange(512)
    u = (2 * (qx + 0.5) / 512 - 1) * tx                             # line of sight at z1: x = u * z1
    s = u * z1 / rho
    sc_ = np.clip(s, -1, 1)
    # part of the disc beyond x = 0 on the side away from its centre
    seg = (np.arccos(np.abs(sc_)) - np.abs(sc_) * np.sqrt(1 - sc_ ** 2)) / math.pi
    want = np.where(s > 0, seg, 1.0 - seg)                          # fraction at x < 0 (occluder side)
    got = h.mean(0)
    band = np.abs(s) < 1.2
    assert band.sum() > 20
    err = np.abs(got[band] - want[band])
    assert err.max() < 0.09 and err.mean() < 0.03


# ---------------------------------------------------------------- temporal

def test_moving_average_closed_form(orc):
    """Static camera, constant far-field input c0, history H: after n frames
    the accumulated colour is c0 + 0.95^n (H - c0) (3.2.3)."""
    lens = synth.Lens()
    scene = plane_scene(40.0, albedo=(0.7, 0.2, 0.4))
    sc = orc.OracleScene(scene)
    cam = synth.look_camera((0, 0, 0), 0, 0, 64, 32)
    gb = orc.gbuffer(sc, cam, lens)
    params = synth.Params(m=1, mask_mode=synth.MASK_ALL)
    npx = 16 * 32
    Hc = np.array([0.1, 0.9, 0.5], np.float32)
    hist = orc.history_zeros(64, 32)
    hist[4 * npx:8 * npx] = np.tile(np.concatenate([Hc, [1.0]]), npx)
    out0 = orc.render_frame(sc, cam, lens, params, gb)
    c0 = out0["resolve"][1][..., :3].reshape(-1, 3)[0].astype(np.float64)
    for n in range(1, 6):
        out = orc.render_frame(sc, dataclasses.replace(cam, frame=n), lens, params, gb, hist_in=hist,
                               prev_cam=cam, prev_lens=lens)
        want = c0 + 0.95 ** n * (Hc - c0)
        np.testing.assert_allclose(out["temporal"][0][..., :3].reshape(-1, 3), np.tile(want, (npx, 1)), atol=2e-6)
        hist = out["hist_out"]


def test_reset_equals_first_frame(orc, small):
    c = small
    cam1 = synth.pan_camera(c["cam"], 0.02)
    gb1 = orc.gbuffer(c["sc"], cam1, c["lens"])
    garbage = np.full_like(c["out"]["hist_out"], 7.0)
    a = orc.render_frame(c["sc"], cam1, c["lens"], c["params"], gb1, hist_in=garbage, prev_cam=c["cam"],
                         prev_lens=c["lens"], reset=True)
    b = orc.render_frame(c["sc"], cam1, c["lens"], c["params"], gb1)
    assert np.array_equal(a["colour"], b["colour"]) and np.array_equal(a["hist_out"], b["hist_out"])


def test_history_reprojection_static_and_pan(orc, small):
    c = small
    out1 = orc.render_frame(c["sc"], dataclasses.replace(c["cam"], frame=1), c["lens"], c["params"], c["gb"],
                            hist_in=c["out"]["hist_out"], prev_cam=c["cam"], prev_lens=c["lens"])
    hw = 128
    valid = c["out"]["mask"].ravel() > 0
    idx = out1["prev_idx"].ravel()
    assert np.array_equal(idx[valid], np.flatnonzero(valid))
    # temporal variance stays non-negative and the blur is the 3x3 binomial
    var = out1["temporal"][1][..., 2]
    assert (var >= 0).all()
    k = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    blur = ndi.correlate(var.astype(np.float64), k, mode="nearest")
    np.testing.assert_allclose(out1["var_blur"], blur, rtol=1e-5, atol=1e-12)


# ---------------------------------------------------------------- reconstruction

def test_zero_variance_weight_keeps_median(orc, small):
    """Eq. (5) with b = 0: the reconstruction returns the median-filtered
    ray-traced colour unchanged (3.2.4)."""
    c = small
    p = dataclasses.replace(c["params"], var_recon_w=0.0)
    out = orc.render_frame(c["sc"], c["cam"], c["lens"], p, c["gb"])
    valid = out["temporal"][0][..., 3] > 0
    assert np.array_equal(out["recon"][valid][:, :3], out["rtmed"][valid][:, :3])


def test_rt_median_is_median_over_valid(small):
    T0 = small["out"]["temporal"][0]
    valid = T0[..., 3] > 0
    hh, hw = valid.shape
    for y, x in list(zip(*np.nonzero(valid)))[::97]:
        for c in range(3):
            vals = []
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy, xx = min(max(y + dy, 0), hh - 1), min(max(x + dx, 0), hw - 1)
                    vals.append(T0[yy, xx, c] if valid[yy, xx] else T0[y, x, c])
            assert small["out"]["rtmed"][y, x, c] == np.float32(np.median(vals))


def test_mip_chain_box_average(small):
    out = small["out"]
    from oracle import mip_dims
    dims = mip_dims(128, 128)
    off = 0
    levels = []
    for w, h in dims:
        levels.append(out["mips"][off:off + w * h * 4].reshape(h, w, 4))
        off += w * h * 4
    m0 = levels[0]
    np.testing.assert_array_equal(m0[..., 3], (out["temporal"][0][..., 3] > 0).astype(np.float32))
    for L in range(1, 4):
        src = levels[L - 1].astype(np.float64)
        want = 0.25 * (src[0::2, 0::2] + src[0::2, 1::2] + src[1::2, 0::2] + src[1::2, 1::2])
        np.testing.assert_allclose(levels[L], want, rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------- estimator

def test_ray_traced_dof_converges_to_lens_integral(orc, small):
    """Cook's distributed ray tracing (3.2.2) is a Monte Carlo estimate of the
    lens integral: against a 64 x 64 stratified quadrature of the aperture the
    RMS error falls roughly as spp^-1/2."""
    c = small
    T0 = c["out"]["resolve"][1][..., 3]
    # silhouette pixels of the foreground bars: partial hit ratio
    cand = np.flatnonzero((T0.ravel() > 0.05) & (T0.ravel() < 0.95))[:48]
    assert cand.size >= 24
    ref = orc.lens_integral(c["sc"], c["cam"], c["lens"], cand, grid=64).astype(np.float64)
    errs = []
    for spp in (1, 4, 16, 64, 256):
        est = orc.pixel_estimate(c["sc"], c["cam"], c["lens"], cand, spp).astype(np.float64)
        errs.append(math.sqrt(((est - ref) ** 2).mean()))
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[1] / 4.0
    assert errs[-1] < 0.03


# ---------------------------------------------------------------- mask dilation (5.3)

def _dilate_pair(orc, small, W, H, lens, m=4):
    cam = dataclasses.replace(small["cam"], width=W, height=H)
    gb = orc.gbuffer(small["sc"], cam, lens)
    p = synth.Params(m=m)
    raw = orc.render_frame(small["sc"], cam, lens, p, gb)
    dil = orc.render_frame(small["sc"], cam, lens, dataclasses.replace(p, mask_mode=synth.MASK_DILATE), gb)
    return raw, dil


def test_mask_dilation_reduces_to_a_max_filter_when_the_radius_is_uniform(orc, small):
    """With at most 3 x 3 tiles every tile's neighbourhood (+-2 tiles) is the
    whole image, so all tiles share one radius R and the dilation is the
    library maximum filter of side 2R + 1 with zeros outside the image."""
    raw, dil = _dilate_pair(orc, small, 96, 64, dataclasses.replace(small["lens"], fnum=0.5))
    td = dil["tile_dil"]
    assert td.shape == (2, 3) and np.all(td == td.flat[0]) and td.flat[0] > 1.0
    R = int(math.ceil(float(td.flat[0])))
    want = ndi.maximum_filter(raw["mask"], size=2 * R + 1, mode="constant", cval=0)
    assert np.array_equal(dil["mask"], want)
    assert (dil["mask"] >= raw["mask"]).all() and dil["n_rays"] > raw["n_rays"]


def test_mask_dilation_only_grows_the_mask(orc, small):
    """Dilation is extensive: every count is at least the adaptive count and
    the ray total only grows (full 256 x 256 workload, radii vary by tile)."""
    raw, dil = _dilate_pair(orc, small, 256, 256, small["lens"])
    assert len(np.unique(dil["tile_dil"])) > 1
    assert (dil["mask"] >= raw["mask"]).all() and dil["n_rays"] >= raw["n_rays"]
    # every pixel dilated from zero has a masked pixel within its tile's radius
    grown = (raw["mask"] == 0) & (dil["mask"] > 0)
    assert grown.any()


def test_mask_dilation_is_identity_without_blur(orc, small):
    """a = 0: every CoC radius is 0, so R = 0 and the mask is unchanged."""
    lens = dataclasses.replace(small["lens"], fnum=math.inf)
    raw, dil = _dilate_pair(orc, small, 64, 48, lens)
    assert np.all(dil["tile_dil"] == 0.0)
    assert np.array_equal(dil["mask"], raw["mask"])


# ---------------------------------------------------------------- final TAA (3.4)

def _taa_plane(hist, W, H):
    import oracle
    o = oracle.taa_offset(W, H)
    return hist[o:o + 4 * W * H].reshape(H, W, 4)


def _raster_plane(hist, W, H):
    import oracle
    o = oracle.raster_taa_offset(W, H)
    return hist[o:o + 4 * W * H].reshape(H, W, 4)


def _post_plane(hist, W, H):
    import oracle
    o = oracle.post_taa_offset(W, H)
    return hist[o:o + W * H].reshape(H // 2, W // 2, 4)


def test_taa_without_history_is_the_composite(orc, small):
    cam, lens, gb = small["cam"], small["lens"], small["gb"]
    off = orc.render_frame(small["sc"], cam, lens, small["params"], gb)
    on = orc.render_frame(small["sc"], cam, lens, dataclasses.replace(small["params"], taa=1), gb)
    assert np.array_equal(on["colour"], off["colour"])
    assert np.array_equal(_taa_plane(on["hist_out"], cam.width, cam.height), on["colour"])


def test_taa_keeps_a_constant_image_whatever_the_history(orc):
    """The history is clamped to the current 3 x 3 range, which is a single
    value on a constant image, so any history leaves the image unchanged."""
    lens = synth.Lens()
    sc = orc.OracleScene(plane_scene(lens.focus))
    cam = synth.look_camera((0, 0, 0), 0, 0, 64, 48)
    p = synth.Params(taa=1)
    gb = orc.gbuffer(sc, cam, lens)
    f0 = orc.render_frame(sc, cam, lens, p, gb)
    assert np.all(f0["colour"] == f0["colour"][0, 0])
    hist = f0["hist_out"].copy()
    rng = np.random.default_rng(5)
    _taa_plane(hist, 64, 48)[...] = rng.uniform(-3.0, 5.0, (48, 64, 4)).astype(np.float32)
    f1 = orc.render_frame(sc, dataclasses.replace(cam, frame=1), lens, p, gb, hist_in=hist, prev_cam=cam,
                          prev_lens=lens)
    assert np.array_equal(f1["colour"], f0["colour"])


def test_taa_onto_its_own_composite_is_identity(orc, small):
    """Static camera, history = the current composite: every pixel reprojects
    onto itself, so the blend returns the composite (up to the bilinear
    weights of a self-reprojection computed in binary32)."""
    cam, lens, gb, p = small["cam"], small["lens"], small["gb"], small["params"]
    f0 = orc.render_frame(small["sc"], cam, lens, p, gb)
    cam1 = dataclasses.replace(cam, frame=1)
    comp1 = orc.render_frame(small["sc"], cam1, lens, p, gb, hist_in=f0["hist_out"], prev_cam=cam, prev_lens=lens)
    hist = f0["hist_out"].copy()
    _taa_plane(hist, cam.width, cam.height)[...] = comp1["colour"]
    t1 = orc.render_frame(small["sc"], cam1, lens, dataclasses.replace(p, taa=1), gb, hist_in=hist, prev_cam=cam,
                          prev_lens=lens)
    np.testing.assert_allclose(t1["colour"], comp1["colour"], atol=1e-4)
    assert not np.array_equal(f0["colour"], comp1["colour"])      # the composite itself changed between frames




def _pan_setup(orc, s, grid_w, z0=10.0, W=64, H=48, seed=9):
    """Pinhole lens (the composite is the G-buffer colour), a seeded random
    colour field over a plane at depth z0 facing the camera, and a second
    camera panned right by exactly s pixel pitches of a grid_w-wide grid at
    that depth."""
    lens = synth.Lens(fnum=math.inf)
    tanx = (lens.sensor * (lens.focus - lens.focal)) / (2.0 * lens.focal * lens.focus)   # half field of view
    cam0 = synth.look_camera((0, 0, 0), 0, 0, W, H)
    cam1 = synth.pan_camera(cam0, s * z0 * 2.0 * tanx / grid_w)
    rng = np.random.default_rng(seed)
    col = np.ones((H, W, 4), np.float32)
    col[..., :3] = rng.uniform(0.0, 1.0, (H, W, 3))
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 2] = -1.0
    gb = orc.GBuffer(col, np.full((H, W), z0, np.float32), nrm)
    sc = orc.OracleScene(plane_scene(z0))
    sc.build_bvh()
    return lens, cam0, cam1, col, gb, sc


def _closed_form(cur, s):
    """(3 x 3 minimum, c + 0.9 (min - c) where x + s is on the grid, c
    elsewhere), RGB; scipy's filter with clamp to edge."""
    from scipy.ndimage import minimum_filter
    mn = minimum_filter(cur[..., :3], size=(3, 3, 1), mode="nearest")
    w = cur.shape[1]
    exp = cur[..., :3].copy()
    exp[:, :w - s] = cur[:, :w - s, :3] + 0.9 * (mn[:, :w - s] - cur[:, :w - s, :3])
    return mn, exp


@pytest.mark.parametrize("stage", [synth.TAA_FINAL, synth.TAA_RASTER])
def test_taa_weight_window_and_reprojection_closed_form(orc, stage):
    """Pixel x of the panned frame sees what pixel x + s saw; the stage's
    history plane holds the 3 x 3 minimum of the new colour field moved s
    pixels right.  Expected: c + 0.9 (min - c) where x + s is on screen, c
    elsewhere.  With a pinhole lens the composite is the resolved raster
    colour, so for the raster stage this also shows in the output."""
    W, H, s = 64, 48, 3
    lens, cam0, cam1, col, gb, sc = _pan_setup(orc, s, W)
    p = synth.Params(taa=stage)
    f0 = orc.render_frame(sc, cam0, lens, p, gb)
    plain = orc.render_frame(sc, cam1, lens, dataclasses.replace(p, taa=0), gb, hist_in=f0["hist_out"],
                             prev_cam=cam0, prev_lens=lens)
    assert np.array_equal(plain["colour"][..., :3], col[..., :3])          # pinhole: composite = G-buffer
    mn, exp = _closed_form(col, s)
    plane_of = _taa_plane if stage == synth.TAA_FINAL else _raster_plane
    hist = f0["hist_out"].copy()
    plane = plane_of(hist, W, H)
    plane[:, s:, :3] = mn[:, :W - s]
    plane[:, :s, :3] = 7.0                                                  # never fetched
    t1 = orc.render_frame(sc, cam1, lens, p, gb, hist_in=hist, prev_cam=cam0, prev_lens=lens)
    np.testing.assert_allclose(t1["colour"][..., :3], exp, rtol=0, atol=2e-4)
    out_plane = plane_of(t1["hist_out"], W, H)
    np.testing.assert_allclose(out_plane[..., :3], exp, rtol=0, atol=2e-4)
    assert np.all(out_plane[..., 3] == 1.0)


def test_post_filter_taa_closed_form(orc):
    """The same construction on the half-res grid of the post-filter output:
    a pan of s half-res pitches, and the post-filter plane of the history set
    to the 3 x 3 minimum of this frame's post-filter output moved s pixels
    right.  The resolved plane is c + 0.9 (min - c) where x + s is on the
    grid, c elsewhere, and keeps the output's 4th channel."""
    W, H, s = 64, 48, 2
    lens, cam0, cam1, col, gb, sc = _pan_setup(orc, s, W // 2)
    p = synth.Params(taa=synth.TAA_POST)
    f0 = orc.render_frame(sc, cam0, lens, p, gb)
    probe = orc.render_frame(sc, cam1, lens, p, gb, hist_in=f0["hist_out"], prev_cam=cam0, prev_lens=lens)
    ppm = probe["ppmed"]
    assert ppm.shape == (H // 2, W // 2, 4) and np.ptp(ppm[..., :3]) > 0.1
    mn, exp = _closed_form(ppm, s)
    hist = f0["hist_out"].copy()
    plane = _post_plane(hist, W, H)
    plane[:, s:, :3] = mn[:, :W // 2 - s]
    plane[:, :s, :3] = 7.0
    t1 = orc.render_frame(sc, cam1, lens, p, gb, hist_in=hist, prev_cam=cam0, prev_lens=lens)
    assert np.array_equal(t1["ppmed"], ppm)                                # the median is upstream of the TAA
    out_plane = _post_plane(t1["hist_out"], W, H)
    np.testing.assert_allclose(out_plane[..., :3], exp, rtol=0, atol=2e-4)
    assert np.array_equal(out_plane[..., 3], ppm[..., 3])


@pytest.mark.parametrize("stage", [synth.TAA_RASTER, synth.TAA_POST, synth.TAA_ALL])
def test_taa_stages_without_history_pass_through(orc, small, stage):
    """Frame 0 (no history): every TAA stage passes its image through, so the
    frame equals the frame without TAA, and each enabled stage's history
    plane holds its input (raster: the G-buffer colour; post-filter: the
    median output)."""
    cam, lens, gb, p = small["cam"], small["lens"], small["gb"], small["params"]
    W, H = cam.width, cam.height
    off = orc.render_frame(small["sc"], cam, lens, p, gb)
    on = orc.render_frame(small["sc"], cam, lens, dataclasses.replace(p, taa=stage), gb)
    for k in ("colour", "mask", "ppmed", "recon", "colr"):
        assert np.array_equal(on[k], off[k]), k
    if stage & synth.TAA_RASTER:
        assert np.array_equal(_raster_plane(on["hist_out"], W, H)[..., :3], gb.colour[..., :3])
    if stage & synth.TAA_POST:
        assert np.array_equal(_post_plane(on["hist_out"], W, H), off["ppmed"])


def test_later_stages_read_the_resolved_images(orc, small):
    """With history, the reduce averages the resolved raster colour (2 x 2
    box of the raster plane, not of the G-buffer), and the composite samples
    the resolved post-filter image: a dark post-filter history darkens the
    output while the median output stays the same."""
    cam, lens, gb, p = small["cam"], small["lens"], small["gb"], small["params"]
    W, H = cam.width, cam.height
    f0 = orc.render_frame(small["sc"], cam, lens, dataclasses.replace(p, taa=synth.TAA_ALL), gb)
    cam1 = synth.pan_camera(cam, 0.02)
    gb1 = orc.gbuffer(small["sc"], cam1, lens)
    t = orc.render_frame(small["sc"], cam1, lens, dataclasses.replace(p, taa=synth.TAA_RASTER), gb1,
                         hist_in=f0["hist_out"], prev_cam=cam, prev_lens=lens)
    r = _raster_plane(t["hist_out"], W, H)
    assert not np.array_equal(r[..., :3], gb1.colour[..., :3])
    box = ((r[0::2, 0::2, :3] + r[0::2, 1::2, :3]) + (r[1::2, 0::2, :3] + r[1::2, 1::2, :3])) * np.float32(0.25)
    assert np.array_equal(t["colr"][..., :3], box)
    hist = f0["hist_out"].copy()
    _post_plane(hist, W, H)[..., :3] = 0.0
    base = orc.render_frame(small["sc"], cam1, lens, dataclasses.replace(p, taa=synth.TAA_POST), gb1,
                            hist_in=f0["hist_out"], prev_cam=cam, prev_lens=lens)
    dark = orc.render_frame(small["sc"], cam1, lens, dataclasses.replace(p, taa=synth.TAA_POST), gb1,
                            hist_in=hist, prev_cam=cam, prev_lens=lens)
    assert np.array_equal(dark["ppmed"], base["ppmed"])
    darker = dark["colour"][..., :3].sum(-1) < base["colour"][..., :3].sum(-1) - 1e-3
    assert darker.mean() > 0.002 and (dark["colour"][..., :3] <= base["colour"][..., :3] + 1e-6).all()


def test_jitter_moves_the_samples_by_the_stated_offset(orc, small):
    """A jitter of a quarter pixel right and down at W x H puts each sample
    where pixel (2x + 1, 2y + 1) of the unjittered 2W x 2H grid has its
    centre, so the G-buffers agree there (up to rounding at silhouettes)."""
    cam, lens, sc = small["cam"], small["lens"], small["sc"]
    j = orc.gbuffer(sc, dataclasses.replace(cam, jitter=(0.25, 0.25)), lens)
    fine = orc.gbuffer(sc, dataclasses.replace(cam, width=2 * cam.width, height=2 * cam.height), lens)
    ref = fine.depth[1::2, 1::2]
    hit = np.isfinite(ref) & np.isfinite(j.depth)
    sky = ~np.isfinite(ref) & ~np.isfinite(j.depth)
    close = (hit & np.isclose(j.depth, ref, rtol=1e-4)) | sky
    assert close.mean() > 0.995 and hit.mean() > 0.3
    plain = orc.gbuffer(sc, cam, lens)
    assert (~np.isclose(plain.depth, ref, rtol=1e-6) & hit).mean() > 0.05   # the jitter did move the samples


def _flat_gbuffer(orc, W, H, z, colour):
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 2] = -1.0
    return orc.GBuffer(np.ascontiguousarray(colour, np.float32), np.full((H, W), z, np.float32), nrm)


@pytest.mark.parametrize("focal", [0.1, 0.3])
def test_prefilter_taps_on_a_quadratic_field(orc, focal):
    """A3 with one CoC everywhere (so every tap weighs the same) on a colour
    field (X/16)^2 of the half-res column X: the 3 x 3 taps at spacing s
    (half the kernel diameter, which is a quarter of the neighbourhood's
    maximum radius but never below sqrt(2)) average to the mean of the
    piecewise-linear interpolation of the field at X - s, X, X + s
    (numpy.interp).  focal 0.1 puts the diameter on its sqrt(2) floor,
    0.3 above it."""
    W, H, z = 64, 48, 40.0
    lens = synth.Lens(focal=focal, fnum=1.0, focus=5.0)
    hw, hh = W // 2, H // 2
    X = np.arange(hw, dtype=np.float64)
    col = np.ones((H, W, 4), np.float32)
    col[..., :3] = np.repeat(((X / 16.0) ** 2).astype(np.float32), 2)[None, :, None]
    gb = _flat_gbuffer(orc, W, H, z, col)
    sc = orc.OracleScene(plane_scene(z))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    o = orc.render_frame(sc, cam, lens, synth.Params(), gb)
    r = o["colr"][..., 3]
    assert np.all(r == r[0, 0]) and r[0, 0] > 0                       # one far-field radius
    Rn = float(o["tile_dil"].max())
    assert np.all(o["tile_dil"] == Rn)
    s = max(Rn * 0.25, math.sqrt(2.0)) * 0.5
    assert (Rn * 0.25 < math.sqrt(2.0)) == (focal == 0.1)
    f = lambda t: np.interp(t, X, (X / 16.0) ** 2)
    inner = slice(3, hw - 4)
    exp = (f(X - s) + f(X) + f(X + s)) / 3.0
    got = o["pre"][4:hh - 4, inner, 0]
    np.testing.assert_allclose(got, np.broadcast_to(exp[inner], got.shape), rtol=0, atol=1e-5)


def _upsample(plane, W, H):
    """Bilinear upsample of a half-res plane to full-res pixel centres (x/2 -
    1/4, y/2 - 1/4), clamp to edge: scipy.ndimage.map_coordinates."""
    from scipy.ndimage import map_coordinates
    yy, xx = np.meshgrid(np.arange(H) * 0.5 - 0.25, np.arange(W) * 0.5 - 0.25, indexing="ij")
    return np.stack([map_coordinates(plane[..., c].astype(np.float64), [yy, xx], order=1, mode="nearest")
                     for c in range(3)], -1)


@pytest.mark.parametrize("literal", [0, 1])
@pytest.mark.parametrize("case", ["far_near_hits", "far_far_hits", "far_all_miss", "near_bright", "near_dim"])
def test_composite_blend_ends(orc, case, literal):
    """A14's blends at their ends, every half-res pixel ray traced (mask mode
    all) and outside the zone of focus.  Far field (eq. 7): when every ray
    hits in front of the focus plane (ratio 1) the output is the upsampled
    reconstruction; when none does (far hits, or misses: ratio 0) it is the
    upsampled post-process image.  Near field: taps all brighter than
    l_spec (bokeh proportion 1) give the post-process image, all dimmer (0)
    the reconstruction.  The G-buffer is a random texture at one depth, so
    the two images differ; the scene decides what the rays see.  With the
    literal reading of the far-field rule (composite_literal) the far-field
    ends swap: ratio 1 gives the post-process image, ratio 0 the
    reconstruction; the near field does not change."""
    W, H = 64, 48
    far = case.startswith("far")
    z = 40.0 if far else 2.0
    plane_z = {"far_near_hits": 2.0, "far_far_hits": 40.0, "far_all_miss": -50.0}.get(case, 2.0)
    lens = synth.Lens(focal=0.1, fnum=1.0, focus=5.0)
    rng = np.random.default_rng(21)
    lo, hi = (1.5, 3.0) if case == "near_bright" else (0.0, 0.5)
    tex = rng.uniform(lo, hi, (H // 4, W // 4, 3)).astype(np.float32)
    col = np.ones((H, W, 4), np.float32)
    col[..., :3] = np.repeat(np.repeat(tex, 4, 0), 4, 1)
    gb = _flat_gbuffer(orc, W, H, z, col)
    sc = orc.OracleScene(plane_scene(plane_z))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    o = orc.render_frame(sc, cam, lens, synth.Params(mask_mode=synth.MASK_ALL, m=4, composite_literal=literal), gb)
    assert np.all(o["mask"] == 4)
    if far:
        assert np.all(o["recon"][..., 3] == (1.0 if case == "far_near_hits" else 0.0))
    rt, pp = _upsample(o["recon"], W, H), _upsample(o["ppmed"], W, H)
    assert np.abs(rt - pp).max() > 0.05                                    # the two images differ
    to_rt = case in ("far_near_hits", "near_dim")
    if far and literal:
        to_rt = not to_rt
    want = rt if to_rt else pp
    np.testing.assert_allclose(o["colour"][..., :3], want, rtol=0, atol=2e-5)


def test_gather_includes_taps_inside_the_radius_and_counts_bright_ones(orc):
    """A4 with one CoC radius R and one depth everywhere: sampleAlpha is the
    same for every tap and every tap is foreground, so the gather is the plain
    mean of the prefiltered image at the nearest texel of each tap whose
    distance R * frac is below R (the outer ring, at distance exactly R, is
    left out: D(0, i) is a strict comparison), and the bokeh proportion is
    the share of those taps brighter than l_spec (Rec. 709 luma).  Tap
    offsets from the ring table (pinned on its own); positions and rounding
    in binary32 as the pass computes them."""
    W, H, z = 64, 48, 40.0
    lens = synth.Lens(focal=0.3, fnum=1.0, focus=5.0)
    params = synth.Params()
    hw, hh = W // 2, H // 2
    X = np.arange(hw, dtype=np.float64)
    col = np.ones((H, W, 4), np.float32)
    col[..., :3] = np.repeat(((X / 16.0) ** 2).astype(np.float32), 2)[None, :, None]
    gb = _flat_gbuffer(orc, W, H, z, col)
    sc = orc.OracleScene(plane_scene(z))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    o = orc.render_frame(sc, cam, lens, params, gb)
    pre = o["pre"]
    R = np.float32(o["tile_dil"].max())
    assert np.all(o["tile_dil"] == R) and np.all(np.abs(pre[..., 3]) == R) and R > 2
    ox, oy, frac = (np.asarray(a, np.float32) for a in orc.gather_rings(lens, params))
    inc = (R * frac) < R
    assert inc.sum() == 49                                    # centre + rings of 8, 16, 24 taps
    luma = (0.2126 * pre[..., 0] + 0.7152 * pre[..., 1]) + 0.0722 * pre[..., 2]
    exp = np.zeros((hh, hw, 3))
    bok = np.zeros((hh, hw))
    for k in np.nonzero(inc)[0]:
        ys = np.arange(hh, dtype=np.float32)[:, None] + oy[k] * R
        xs = np.arange(hw, dtype=np.float32)[None, :] + ox[k] * R
        iy = np.clip(np.floor(ys + np.float32(0.5)).astype(int), 0, hh - 1)
        ix = np.clip(np.floor(xs + np.float32(0.5)).astype(int), 0, hw - 1)
        iy, ix = np.broadcast_arrays(iy, ix)
        exp += pre[iy, ix, :3]
        bok += luma[iy, ix] > params.l_spec
    n = float(inc.sum())
    np.testing.assert_allclose(o["gather"][..., :3], exp / n, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(o["gather"][..., 3], bok / n, rtol=0, atol=1e-6)
    assert 0.0 < o["gather"][..., 3].mean() < 1.0             # both kinds of tap occur


def test_reconstruction_keeps_a_linear_field_whatever_b(orc):
    """A13 beyond b = 0.  On a colour field linear in x, a box-averaged mip
    level holds the field at each texel's footprint centre, so the bilinear
    sample at a tap's mip coordinates ((x + 1/2) 2^-L - 1/2) is the field at
    the tap itself, on either level; over the symmetric rings the taps then
    average to the centre value, and with every tap valid the reconstruction
    returns its median input unchanged for any blend factor b.  The field is
    put into the ray-traced image through the history: a near plane of one
    colour c hit by every ray, static camera (the near field reprojects each
    pixel onto itself), so the temporal stage gives c + 0.95 (H - c) with H
    the history's near colour, here linear in x; the history's luma moments
    force a large variance, so b sits at its 0.9 cap.  The temporal CoC is
    uniform only to rounding, and an outer-ring tap lies exactly at the
    radius, so a neighbour whose CoC is a few ulps smaller rejects it; the
    expected value therefore takes the mean over the taps that pass the
    rejection rule: centre + b * slope * R * mean(ox over valid taps), which
    is the centre itself when every tap passes."""
    W, H, z = 128, 96, 2.0
    hw, hh = W // 2, H // 2
    np_ = hw * hh
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    col = np.full((H, W, 4), 0.5, np.float32)
    gb = _flat_gbuffer(orc, W, H, z, col)
    sc = orc.OracleScene(plane_scene(z))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    p = synth.Params(mask_mode=synth.MASK_ALL, m=4)
    f0 = orc.render_frame(sc, cam, lens, p, gb)
    hist = f0["hist_out"].copy()
    X = np.arange(hw, dtype=np.float32)
    A = hist[:4 * np_].reshape(hh, hw, 4)
    A[..., :3] = (np.float32(0.2) + np.float32(0.01) * X)[None, :, None]
    A[..., 3] = 1.0                                    # hit ratio: near field only
    Cp = hist[8 * np_:12 * np_].reshape(hh, hw, 4)
    Cp[..., 2] = 0.0                                   # luma mean
    Cp[..., 3] = 1.0                                   # luma second moment
    f1 = orc.render_frame(sc, dataclasses.replace(cam, frame=1), lens, p, gb, hist_in=hist, prev_cam=cam,
                          prev_lens=lens)
    assert np.all(f1["prev_idx"] == np.arange(np_).reshape(hh, hw))   # each pixel onto itself
    assert np.all(f1["temporal"][0][..., 3] > 0)                      # every pixel ray traced
    med, rec = f1["rtmed"], f1["recon"]
    step = np.diff(med[..., 0], axis=1)                # the median input is linear in x
    assert np.abs(step - step.mean()).max() < 1e-5 and abs(step.mean()) > 1e-3
    bb = np.clip(f1["var_blur"] * p.var_recon_w, 0.0, p.b_max)
    assert bb.min() > 0.5                              # b far from 0
    ct = f1["temporal"][1][..., 0]                     # temporal CoC (full-res diameter)
    lod = np.clip(ct * p.lod_scale, 0.0, p.lod_max)
    assert lod.min() > 1.0 and np.any(lod % 1.0 > 0.1)  # two mip levels above the finest, blended
    R = float(ct.max()) * 0.25                         # tap radius
    m = int(math.ceil(R)) + 9                          # taps and coarsest texels stay inside
    assert hh - 2 * m > 2 and hw - 2 * m > 2
    inner = (slice(m, hh - m), slice(m, hw - m))
    ox, oy, frac = orc.gather_rings(synth.Lens(), synth.Params())
    ys, xs = np.mgrid[m:hh - m, m:hw - m]
    Rr = ct[ys, xs].astype(np.float32) * np.float32(0.25)          # per-pixel tap radius
    sx = xs[..., None].astype(np.float32) + ox[None, None, :] * Rr[..., None]
    sy = ys[..., None].astype(np.float32) + oy[None, None, :] * Rr[..., None]
    ix = np.clip(np.floor(sx + np.float32(0.5)).astype(int), 0, hw - 1)
    iy = np.clip(np.floor(sy + np.float32(0.5)).astype(int), 0, hh - 1)
    valid = ~(ct[iy, ix] * np.float32(0.25) < Rr[..., None] * frac[None, None, :])
    assert valid.sum(axis=-1).min() >= 81 - 32                      # at most the outer ring drops
    shift = (ox[None, None, :].astype(np.float64) * valid).sum(-1) / valid.sum(-1) * Rr
    exp = med[inner][..., :3] + (bb[inner] * step.mean() * shift)[..., None]
    np.testing.assert_allclose(rec[inner][..., :3], exp, rtol=0, atol=2e-5)


@pytest.mark.parametrize("field", ["near", "far"])
def test_temporal_reprojection_under_a_pan(orc, field):
    """A12 under camera motion.  The camera pans right by exactly s half-res
    pitches at the depth of a plane facing it, so the point seen at half-res
    pixel x was seen at x + s: each pixel centre reprojects to the middle of
    that pixel, and a reprojection off screen has no history.  The history is
    built by hand (seeded random near and far colours, age 1), and every
    pixel shoots m rays.  A plane nearer than the focus ramp makes every hit near field: the
    G-buffer reprojection (prev_idx) is x + s and the temporal colour is the
    exponential average c + alpha_m (A[x + s] - c) of this frame's near mean
    with the history's near colour, alpha_m the weight during motion.  A
    plane beyond the ramp makes every hit far field: the far field is
    reprojected through the mean far hit position, which lies on the plane
    but off the pixel's centre line by the mean of its lens samples; the
    texel it lands on comes from a pinhole projection into the previous
    camera computed here in binary64 (coordinates within 1e-4 of a texel
    edge skipped), mostly x + s, and the temporal colour averages the far
    mean with the history's far colour there.  Without a history texel the
    temporal colour is this frame's mean.  Age counts up from the history's."""
    W, H, s = 128, 96, 3
    hw, hh = W // 2, H // 2
    np_ = hw * hh
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    z = 2.0 if field == "near" else 6.0
    tanx = (lens.sensor * (lens.focus - lens.focal)) / (2.0 * lens.focal * lens.focus)
    cam0 = synth.look_camera((0, 0, 0), 0, 0, W, H)
    cam1 = synth.pan_camera(cam0, s * z * 2.0 * tanx / hw)
    gb = _flat_gbuffer(orc, W, H, z, np.full((H, W, 4), 0.5, np.float32))
    sc = orc.OracleScene(plane_scene(z))
    sc.build_bvh()
    p = synth.Params(mask_mode=synth.MASK_ALL, m=4)
    hist = orc.history_zeros(W, H)
    rng = np.random.default_rng(5)
    A = hist[:4 * np_].reshape(hh, hw, 4)
    B = hist[4 * np_:8 * np_].reshape(hh, hw, 4)
    A[..., :3] = rng.uniform(0.0, 1.0, (hh, hw, 3))
    A[..., 3] = 1.0 if field == "near" else 0.0
    B[..., :3] = rng.uniform(0.0, 1.0, (hh, hw, 3))
    B[..., 3] = 1.0
    f1 = orc.render_frame(sc, cam1, lens, p, gb, hist_in=hist, prev_cam=cam0, prev_lens=lens)
    X = np.arange(hw)[None, :].repeat(hh, 0)
    Y = np.arange(hh)[:, None].repeat(hw, 1)
    on = X + s < hw
    assert np.array_equal(f1["prev_idx"], np.where(on, Y * hw + X + s, -1))
    T0 = f1["temporal"][0]
    assert np.all(T0[..., 3] == 1.0)                                    # every pixel traced
    a = np.float32(p.alpha_motion)
    if field == "near":
        cur = f1["resolve"][0][..., :3]
        py, px, got = Y, X + s, on
        Hc = A[..., :3]
    else:
        cur = f1["resolve"][1][..., :3]
        fp = f1["resolve"][3]                                            # mean far hit position, validity
        assert np.all(fp[on][:, 3] == 1.0) and np.allclose(fp[on][:, 2], z, rtol=0, atol=1e-5)
        e = fp[..., :3].astype(np.float64) - np.asarray(cam0.pos, np.float64)
        ex, ey, ez = (e @ np.asarray(v, np.float64) for v in (cam0.right, cam0.up, cam0.fwd))
        u = ((ex / ez) / tanx + 1.0) * 0.5 * hw
        w = (1.0 - (ey / ez) / (tanx * H / W)) * 0.5 * hh
        px, py = np.floor(u).astype(int), np.floor(w).astype(int)
        clear = (np.abs(u - np.round(u)) > 1e-4) & (np.abs(w - np.round(w)) > 1e-4)
        got = on & clear & (px >= 0) & (px < hw) & (py >= 0) & (py < hh)
        assert got.sum() > 0.95 * on.sum() and np.mean((px == X + s) & (py == Y)) > 0.8
        Hc = B[..., :3]
        off = clear & ((px >= hw) | (py < 0) | (py >= hh))
        assert off.sum() >= s * hh - hh // 4
        np.testing.assert_allclose(T0[off][:, :3], cur[off], rtol=0, atol=1e-6)   # no history: this frame
    prev = Hc[np.clip(py, 0, hh - 1), np.clip(px, 0, hw - 1)]
    exp = (cur + (prev - cur) * a).astype(np.float32)
    np.testing.assert_allclose(T0[got][:, :3], exp[got], rtol=0, atol=1e-6)
    assert np.ptp(T0[got][:, :3]) > 0.3                                  # the history field shows through
    if field == "near":
        np.testing.assert_allclose(T0[~on][:, :3], cur[~on], rtol=0, atol=1e-6)   # no history: this frame
    hb = f1["hist_out"][4 * np_:8 * np_].reshape(hh, hw, 4)
    assert np.all(hb[on][:, 3] == 2.0)


def test_temporal_merge_of_mixed_fields_static(orc):
    """A12's hit-ratio merge with both fields present.  A plane exactly at the
    focus distance puts every ray at the middle of the near/far ramp (near
    weight 1/2), and all rays of a pixel meet at its focus point, so with a
    static camera both fields reproject onto the pixel itself and this
    frame's hit ratio is 1/2.  Hand-set history: near colour 1, far colour 0,
    accumulated hit ratio 1, near CoC 8, far CoC 2, luma moments 1/2 and 1/2.
    With history weight 0.95 and this frame's colour c (the same in both
    fields: one plane), CoC ~0 and luma l:
        near 0.05 c + 0.95, far 0.05 c, hit ratio 0.5 + 0.5 * 0.95 = 0.975,
        colour = far + 0.975 (near - far) = 0.05 c + 0.92625,
        CoC = 1.9 + 0.975 (7.6 - 1.9) = 7.4575,
        mu1 = 0.05 l + 0.475, mu2 = 0.05 l^2 + 0.475, variance mu2 - mu1^2.
    A swapped merge would give 0.05 c + 0.02375, and merging by this frame's
    hit ratio (the rule during motion) 0.05 c + 0.475."""
    W, H = 128, 96
    hw, hh = W // 2, H // 2
    np_ = hw * hh
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    z = lens.focus
    cam0 = synth.look_camera((0, 0, 0), 0, 0, W, H)
    cam1 = dataclasses.replace(cam0, frame=1)
    gb = _flat_gbuffer(orc, W, H, z, np.full((H, W, 4), 0.5, np.float32))
    sc = orc.OracleScene(plane_scene(z))
    sc.build_bvh()
    p = synth.Params(mask_mode=synth.MASK_ALL, m=4)
    assert p.alpha == pytest.approx(0.95)
    hist = orc.history_zeros(W, H)
    A = hist[:4 * np_].reshape(hh, hw, 4)
    B = hist[4 * np_:8 * np_].reshape(hh, hw, 4)
    C = hist[8 * np_:12 * np_].reshape(hh, hw, 4)
    A[...] = 1.0
    B[..., :3] = 0.0
    B[..., 3] = 1.0
    C[...] = (8.0, 2.0, 0.5, 0.5)
    f1 = orc.render_frame(sc, cam1, lens, p, gb, hist_in=hist, prev_cam=cam0, prev_lens=lens)
    assert np.array_equal(f1["prev_idx"], np.arange(np_).reshape(hh, hw))
    res = f1["resolve"]
    np.testing.assert_allclose(res[1][..., 3], 0.5, rtol=0, atol=1e-5)        # this frame's hit ratio
    c = res[0][..., :3].astype(np.float64)
    np.testing.assert_allclose(res[1][..., :3], c, rtol=0, atol=1e-6)          # one plane: same colour
    T0, T1 = f1["temporal"]
    col = 0.05 * c + 0.92625
    np.testing.assert_allclose(T0[..., :3], col, rtol=0, atol=2e-5)
    np.testing.assert_allclose(T1[..., 0], 7.4575, rtol=0, atol=1e-4)
    np.testing.assert_allclose(T1[..., 1], 0.975, rtol=0, atol=1e-5)
    l = col @ np.array([0.2126, 0.7152, 0.0722])
    mu1, mu2 = 0.05 * l + 0.475, 0.05 * l * l + 0.475
    np.testing.assert_allclose(T1[..., 2], np.maximum(mu2 - mu1 * mu1, 0.0), rtol=0, atol=2e-5)
    assert T1[..., 2].min() > 0.1


def _z_for_radius(orc, lens, W, r):
    """Near-field depth whose half-res CoC radius (diameter / 4) is r, by
    bisection on the oracle's CoC (decreasing in depth before the focus)."""
    lo, hi = 1e-3, lens.focus
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if orc.coc(lens, W, mid) / 4.0 > r:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _two_region_gbuffer(orc, W, H, b, z1, z2, c1, c2):
    """Full-res G-buffer: depth z1 and colour c1 left of full-res column 2b,
    z2 and c2 from there on; normals face the camera."""
    depth = np.full((H, W), z1, np.float32)
    depth[:, 2 * b:] = z2
    col = np.ones((H, W, 4), np.float32)
    col[:, :2 * b, :3] = c1
    col[:, 2 * b:, :3] = c2
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 2] = -1.0
    return orc.GBuffer(col, depth, nrm)


def test_prefilter_weights_across_a_coc_step(orc):
    """A3 at differing CoCs.  Two near-field regions meet at half-res column b:
    CoC radius 8 on the left, 6 on the right.  The dilated maximum radius 8
    sets the kernel diameter to 8/4 = 2 and the tap spacing to 1, so the 3 x 3
    taps sit on texel centres.  Next to the step, 6 taps share the centre's
    radius (weight 1) and 3 differ by 2 (weight 1/(1 + 2) = 1/3):
    (6 c1 + c2) / 7 left of it, (c1 + 6 c2) / 7 right of it, and the plain
    region colour one texel further away."""
    W, H, b = 128, 64, 32
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    z1, z2 = _z_for_radius(orc, lens, W, 8.0), _z_for_radius(orc, lens, W, 6.0)
    c1, c2 = np.array([0.9, 0.2, 0.4], np.float32), np.array([0.1, 0.7, 0.3], np.float32)
    gb = _two_region_gbuffer(orc, W, H, b, z1, z2, c1, c2)
    sc = orc.OracleScene(plane_scene(z1))
    out = orc.render_frame(sc, synth.look_camera((0, 0, 0), 0, 0, W, H), lens, synth.Params(), gb)
    r = out["colr"][..., 3]
    np.testing.assert_allclose(r[:, :b], -8.0, rtol=0, atol=1e-4)           # near field: negative radius
    np.testing.assert_allclose(r[:, b:], -6.0, rtol=0, atol=1e-4)
    np.testing.assert_allclose(out["colr"][:, :b, :3], np.broadcast_to(c1, (H // 2, b, 3)), rtol=0, atol=1e-6)
    pre = out["pre"][..., :3].astype(np.float64)
    want = {b - 2: c1, b - 1: (6.0 * c1 + c2) / 7.0, b: (c1 + 6.0 * c2) / 7.0, b + 1: c2}
    for x, v in want.items():
        np.testing.assert_allclose(pre[:, x], np.broadcast_to(v, (H // 2, 3)), rtol=0, atol=2e-5)


def _z_far_for_radius(orc, lens, W, r):
    """Far-field depth whose half-res CoC radius is r (CoC rising with depth
    beyond the focus)."""
    lo, hi = lens.focus, 1e6
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if orc.coc(lens, W, mid) / 4.0 < r:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _gather_taps(orc, lens, params, x, y, Rn, hw, hh):
    """Columns, rows and ring numbers (0 = centre .. 4 = rim) of the 81 taps
    of half-res pixel (x, y) at radius Rn, nearest texel."""
    ox, oy, frac = orc.gather_rings(lens, params)
    sx = np.float32(x) + ox * np.float32(Rn)
    sy = np.float32(y) + oy * np.float32(Rn)
    col = np.clip(np.floor(sx + np.float32(0.5)).astype(int), 0, hw - 1)
    row = np.clip(np.floor(sy + np.float32(0.5)).astype(int), 0, hh - 1)
    return col, row, np.round(frac * 4).astype(int)


def _luma(c):
    return c @ np.array([0.2126, 0.7152, 0.0722])


def test_gather_foreground_bleeds_over_a_sharp_background(orc):
    """A4 at differing CoCs and depths: eq. (1) as scatter-as-gather.  Left of
    half-res column b a near, strongly blurred foreground (radius 8, bright:
    luma above l_spec), right of it a sharp background (radius 0.4) more than
    the depth range behind it.  For a background centre next to the step
    (dilated radius 8: rings at distances 0, 2, 4, 6, 8), a foreground tap
    counts when its own radius 8 exceeds its distance (rings 1-3), with
    sampleAlpha 1 / 8^2; a background tap at the centre's depth counts only
    at distance 0 (radius 0.4), with sampleAlpha 1 / max(0.4, 1/2)^2 = 4.
    Colour = (4 c + sum over the foreground taps of f / 64) / (4 + n_f / 64)
    on the prefiltered colours; the bokeh share is the foreground's weight
    fraction.  Every pixel of the row agrees."""
    W, H, b = 128, 64, 32
    hw, hh = W // 2, H // 2
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    p = synth.Params()
    z1, z2 = _z_for_radius(orc, lens, W, 8.0), _z_for_radius(orc, lens, W, 0.4)
    assert z2 - z1 > p.depth_range
    c1, c2 = np.array([3.0, 2.5, 2.0], np.float32), np.array([0.2, 0.4, 0.3], np.float32)
    gb = _two_region_gbuffer(orc, W, H, b, z1, z2, c1, c2)
    out = orc.render_frame(orc.OracleScene(plane_scene(z1)), synth.look_camera((0, 0, 0), 0, 0, W, H), lens, p, gb)
    r, pre, gat = out["colr"][..., 3], out["pre"][..., :3].astype(np.float64), out["gather"]
    np.testing.assert_allclose(r[:, :b], -8.0, rtol=0, atol=1e-4)
    np.testing.assert_allclose(r[:, b:], -0.4, rtol=0, atol=1e-4)
    assert np.all(out["tile_dil"] == out["tile_dil"].max())
    Rn = float(out["tile_dil"].max())
    assert abs(Rn - 8.0) < 1e-4
    for x in (b, b + 1, b + 3, b + 5):
        for y in (3, hh // 2, hh - 2):
            col, row, ring = _gather_taps(orc, lens, p, x, y, Rn, hw, hh)
            fg = (col < b) & (ring >= 1) & (ring <= 3)
            w = np.where(fg, 1.0 / 64.0, 0.0)
            w[ring == 0] = 4.0
            assert fg.sum() > 0
            taps = pre[row, col]
            exp = (w[:, None] * taps).sum(0) / w.sum()
            np.testing.assert_allclose(gat[y, x, :3], exp, rtol=0, atol=2e-5)
            share = w[_luma(taps) > p.l_spec].sum() / w.sum()
            assert abs(gat[y, x, 3] - share) < 2e-5 and 0.0 < share < 1.0


def test_gather_background_needs_the_centre_radius(orc):
    """A4: a background tap counts only where the smaller of its radius and
    the centre's exceeds its distance.  Left of half-res column b a mildly
    blurred near foreground (radius 2), right of it a strongly blurred far
    background (radius 6).  For a foreground centre three or four texels from
    the step (dilated radius 6: rings at 0, 1.5, 3, 4.5, 6), the background
    taps on rings 2-3 have radius 6 beyond their distance but the centre's
    2 is not, so none counts; foreground taps count on rings 0-1 (radius 2 >
    1.5), which stay left of the step.  Colour = mean of the prefiltered
    colour over those 9 taps (one sampleAlpha 1/4 for all)."""
    W, H, b = 256, 64, 64
    hw, hh = W // 2, H // 2
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    p = synth.Params()
    z1, z2 = _z_for_radius(orc, lens, W, 2.0), _z_far_for_radius(orc, lens, W, 6.0)
    c1, c2 = np.array([0.8, 0.3, 0.1], np.float32), np.array([0.1, 0.5, 0.9], np.float32)
    gb = _two_region_gbuffer(orc, W, H, b, z1, z2, c1, c2)
    out = orc.render_frame(orc.OracleScene(plane_scene(z1)), synth.look_camera((0, 0, 0), 0, 0, W, H), lens, p, gb)
    r, pre, gat = out["colr"][..., 3], out["pre"][..., :3].astype(np.float64), out["gather"]
    np.testing.assert_allclose(r[:, :b], -2.0, rtol=0, atol=1e-4)
    np.testing.assert_allclose(r[:, b:], 6.0, rtol=0, atol=1e-4)
    Rn = float(out["tile_dil"].max())
    assert abs(Rn - 6.0) < 1e-4
    for x in (b - 3, b - 4):
        for y in (3, hh // 2):
            assert out["tile_dil"][y // p.tile, x // p.tile] == Rn             # dilated radius at the centre
            col, row, ring = _gather_taps(orc, lens, p, x, y, Rn, hw, hh)
            use = ring <= 1
            assert np.all(col[use] < b) and np.any((col >= b) & (ring >= 2) & (ring <= 3))
            exp = pre[row[use], col[use]].mean(0)
            np.testing.assert_allclose(gat[y, x, :3], exp, rtol=0, atol=2e-5)


def test_reconstruction_mips_weight_by_validity(orc):
    """A13 where ray-traced and empty pixels mix.  Only even half-res columns
    are ray traced (their G-buffer depth is a near plane, out of focus; odd
    columns sit at the focus distance, and with eq. (2)'s scale s = 0 only
    out-of-focus near pixels get a ray), and the ray-traced colour is linear
    in x, f(x), put in through the history as in the b > 0 pin above.  A mip
    texel of level L >= 1 then averages valid children at columns
    2^L X, 2^L X + 2, ...: its validity is 1/2 and its validity-normalised
    colour f(2^L X + 2^(L-1) - 1), so every bilinear sample at a tap's mip
    coordinates reads f(x_tap - 1/2) with weight 1/2 on both levels: the
    validity weighting moves the field by half a pixel.  With b at its cap,
    the median equal to the centre (its empty neighbours are replaced by the
    centre) and only taps on ray-traced texels that pass the CoC rejection
    counted: reconstruction = f(x) + b * slope * (R * mean(ox over valid
    taps) - 1/2) at every even column away from the borders."""
    W, H = 128, 96
    hw, hh = W // 2, H // 2
    np_ = hw * hh
    lens = synth.Lens(focal=0.15, fnum=1.0, focus=5.0)
    depth = np.full((H, W), lens.focus, np.float32)
    for X in range(0, hw, 2):
        depth[:, 2 * X:2 * X + 2] = 2.0
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 2] = -1.0
    gb = orc.GBuffer(np.full((H, W, 4), 0.5, np.float32), depth, nrm)
    sc = orc.OracleScene(plane_scene(2.0))
    sc.build_bvh()
    cam = synth.look_camera((0, 0, 0), 0, 0, W, H)
    p = synth.Params(s=0.0)
    f0 = orc.render_frame(sc, cam, lens, p, gb)
    hist = f0["hist_out"].copy()
    X = np.arange(hw, dtype=np.float32)
    A = hist[:4 * np_].reshape(hh, hw, 4)
    A[..., :3] = (np.float32(0.2) + np.float32(0.01) * X)[None, :, None]
    A[..., 3] = 1.0
    hist[4 * np_ + 3:8 * np_:4] = 1.0                     # age: the history is valid everywhere
    C = hist[8 * np_:12 * np_].reshape(hh, hw, 4)
    C[..., 2] = 0.0
    C[..., 3] = 1.0
    f1 = orc.render_frame(sc, dataclasses.replace(cam, frame=1), lens, p, gb, hist_in=hist, prev_cam=cam,
                          prev_lens=lens)
    traced = f1["temporal"][0][..., 3] > 0
    assert np.array_equal(traced, np.broadcast_to(X % 2 == 0, (hh, hw)))
    med, rec = f1["rtmed"], f1["recon"]
    even = med[:, 0::2, 0]
    step = np.diff(even, axis=1).mean() / 2.0                          # slope per half-res pixel
    assert abs(step) > 1e-3 and np.abs(np.diff(even, axis=1) - 2 * step).max() < 1e-5
    bb = np.clip(f1["var_blur"] * p.var_recon_w, 0.0, p.b_max)
    ct = f1["temporal"][1][..., 0]
    lod = np.clip(ct * p.lod_scale, 0.0, p.lod_max)
    assert bb[traced].min() == np.float32(p.b_max) and lod[traced].min() > 1.0   # b capped; mip levels >= 1
    R = float(ct[traced].max()) * 0.25
    m = int(math.ceil(R)) + 9
    ox, oy, frac = orc.gather_rings(synth.Lens(), synth.Params())
    checked = 0
    for y in range(m, hh - m):
        for x in range(m + (m % 2), hw - m, 2):
            Rr = np.float32(ct[y, x]) * np.float32(0.25)
            sx = np.float32(x) + ox * Rr
            sy = np.float32(y) + oy * Rr
            ix = np.floor(sx + np.float32(0.5)).astype(int)
            iy = np.floor(sy + np.float32(0.5)).astype(int)
            valid = traced[iy, ix] & ~(ct[iy, ix] * np.float32(0.25) < Rr * frac)
            shift = float(Rr) * (ox.astype(np.float64) * valid).sum() / valid.sum() - 0.5
            exp = med[y, x, :3] + bb[y, x] * step * shift
            np.testing.assert_allclose(rec[y, x, :3], exp, rtol=0, atol=2e-5)
            checked += 1
    assert checked > 100


def test_temporal_far_position_filled_from_neighbours(orc):
    """A12's fill of a missing far hit position.  Far-field strips (z = 7,
    beyond the focus ramp) each exactly one half-res pixel wide cover the
    even columns, with sky between them; a small aperture (f/4) keeps every
    pixel's rays inside its own footprint, so even columns hit only strip
    and odd columns only sky.  A miss adds no far position, so an odd pixel
    has none and takes the mean of its valid 3 x 3 neighbours' (the six on
    the even columns beside it), which lies on the strip plane over its own
    centre and so, with a static camera, reprojects onto the pixel itself.
    With the history's hit ratio 0 (the merge then keeps the far field) its
    temporal colour is sky + 0.95 (B[y, x] - sky) for a seeded random far
    history B; without the fill it would be the sky colour.  The camera sits
    away from the world origin, so a position pulled towards the origin (a
    fill that counted empty neighbours as zeros) lands on another texel."""
    W, H = 128, 96
    hw, hh = W // 2, H // 2
    np_ = hw * hh
    lens = synth.Lens(focal=0.15, fnum=4.0, focus=5.0)
    tanx = (lens.sensor * (lens.focus - lens.focal)) / (2.0 * lens.focal * lens.focus)
    z = 7.0
    c0 = (0.4, 0.3, -2.0)                                              # camera position
    quads = []
    for X in range(0, hw, 2):
        x0 = c0[0] + (X * 2.0 / hw - 1.0) * tanx * z
        x1 = c0[0] + ((X + 1) * 2.0 / hw - 1.0) * tanx * z
        zw = c0[2] + z
        quads.append(synth.quad((x0, -50.0, zw), (x0, 50.0, zw), (x1, 50.0, zw), (x1, -50.0, zw)))
    v = np.concatenate(quads).astype(np.float32)
    sky = (0.55, 0.70, 0.95)
    sc = orc.OracleScene(synth.Scene(v, np.full((len(v), 3), 0.5, np.float32), sky=sky))
    sc.build_bvh()
    cam = synth.look_camera(c0, 0, 0, W, H)
    gb = _flat_gbuffer(orc, W, H, z, np.full((H, W, 4), 0.5, np.float32))
    p = synth.Params(mask_mode=synth.MASK_ALL, m=4)
    hist = orc.history_zeros(W, H)
    B = hist[4 * np_:8 * np_].reshape(hh, hw, 4)
    B[..., :3] = np.random.default_rng(11).uniform(0.0, 1.0, (hh, hw, 3))
    B[..., 3] = 1.0                                                     # age
    f1 = orc.render_frame(sc, dataclasses.replace(cam, frame=1), lens, p, gb, hist_in=hist, prev_cam=cam,
                          prev_lens=lens)
    res = f1["resolve"]
    odd = np.broadcast_to(np.arange(hw) % 2 == 1, (hh, hw))
    assert np.all(res[3][..., 3][~odd] == 1.0) and np.all(res[3][..., 3][odd] == 0.0)   # own far position or none
    assert np.all(res[1][..., 3] == 0.0)                                # hit ratio 0: no near hits
    np.testing.assert_allclose(res[1][odd][:, :3], np.broadcast_to(sky, (odd.sum(), 3)), rtol=0, atol=1e-6)
    T0 = f1["temporal"][0]
    inner = np.zeros((hh, hw), bool)
    inner[1:-1, 1:-1] = True
    sel = odd & inner
    exp = np.asarray(sky, np.float32) + (B[..., :3] - np.asarray(sky, np.float32)) * np.float32(0.95)
    np.testing.assert_allclose(T0[sel][:, :3], exp[sel], rtol=0, atol=2e-6)
    assert sel.sum() > 1000
