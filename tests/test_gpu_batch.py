"""Batched launches (several sessions' frames per launch) through the C ABI.

Every item of a batch must come out bit-identical to the same frame rendered
alone by dof_render_frame: colour, mask, history, stats and every
intermediate plane.  One item is also compared with the CPU oracle to the
usual parity bar (index work exact, colour within 1e-3), and a batch run
captured in a HIP graph is replayed several times against eager results."""

import dataclasses

import numpy as np
import pytest

from paper_2210_06158_amd import synth

pytestmark = pytest.mark.gpu

COLOUR_TOL = 1e-3
PLANES = ("colr", "zn", "tile_max", "tile_dil", "pre", "gather", "ppmed", "prev_idx", "queue", "ray_base",
          "ray_hit", "ray_t", "ray_col", "ray_pos", "resolve", "temporal", "var_blur", "rtmed", "mips", "recon")


@pytest.fixture(scope="module")
def sess(orc):
    """Four sessions: different scenes, sizes and apertures (m = 4 shared)."""
    import torch
    from paper_2210_06158_amd import dof
    torch.cuda.set_device(0)
    small, cam_s, lens_s, params = synth.scene_small()
    small2, cam_2, _, _ = synth.scene_small(seed=synth.BASE_SEED + 1777)
    grass, cams_g, lens_g, _ = synth.scene_1080p(seed=synth.BASE_SEED + 5000, n_spheres=64, n_blades=3000,
                                                 width=320, height=180)
    hexa = dataclasses.replace(lens_s, fnum=2.0, blades=6, blade_rot=0.3)
    spec = [
        (small, cam_s, lens_s),
        (small2, dataclasses.replace(cam_2, width=202, height=118), hexa),
        (grass, cams_g[0], lens_g),
        (small, dataclasses.replace(synth.pan_camera(cam_s, 0.05), width=130, height=66), lens_s),
    ]
    scenes = {}
    out = []
    for scene, cam, lens in spec:
        key = id(scene)
        if key not in scenes:
            gs = dof.Scene(scene)
            gs.build_bvh()
            osc = orc.OracleScene(scene)
            osc.build_bvh()
            scenes[key] = (gs, osc)
        gs, osc = scenes[key]
        gb = orc.gbuffer(osc, cam, lens)
        g = (torch.from_numpy(gb.colour).cuda(), torch.from_numpy(gb.depth).cuda(), torch.from_numpy(gb.normal).cuda())
        out.append(dict(scene=scene, gs=gs, osc=osc, cam=cam, lens=lens, gb=gb, g=g))
    torch.cuda.synchronize()
    return dict(torch=torch, dof=dof, params=params, items=out)


def grab(torch, fr, hout):
    torch.cuda.synchronize()
    d = fr.debug()
    d["colour"] = fr.colour.cpu().numpy()
    d["mask"] = fr.mask.cpu().numpy()
    d["stats"] = fr.stats.cpu().numpy()
    d["hist_out"] = hout.cpu().numpy()
    return d


def render_alone(sess, hist_in=None, prev=None):
    torch, dof = sess["torch"], sess["dof"]
    res = []
    for k, it in enumerate(sess["items"]):
        cam = it["cam"]
        fr = dof.Frame(cam.width, cam.height, sess["params"], ray_records=True)
        hout = dof.history_alloc(cam.width, cam.height)
        hin = hist_in[k] if hist_in is not None else None
        pc = prev[k] if prev is not None else None
        fr.render(it["gs"], cam, it["lens"], it["g"], hin, hout, prev_cam=pc, prev_lens=it["lens"])
        res.append(grab(torch, fr, hout))
    return res


def make_frames(sess):
    dof = sess["dof"]
    frs, houts = [], []
    for it in sess["items"]:
        cam = it["cam"]
        frs.append(dof.Frame(cam.width, cam.height, sess["params"], ray_records=True))
        houts.append(dof.history_alloc(cam.width, cam.height))
    return frs, houts


def batch_items(sess, frs, houts, hist_in=None, prev=None):
    items = []
    for k, it in enumerate(sess["items"]):
        hin = hist_in[k] if hist_in is not None else None
        pc = prev[k] if prev is not None else None
        items.append(frs[k].item(it["gs"], it["cam"], it["lens"], it["g"], hin, houts[k], prev_cam=pc,
                                 prev_lens=it["lens"]))
    return items


def same(a, b, label):
    m = b["mask"] > 0
    for key in ("colour", "mask", "hist_out") + PLANES:
        x, y = np.asarray(a[key]), np.asarray(b[key])
        if key == "resolve":      # written for masked pixels only
            x, y = np.ascontiguousarray(x[:, m]), np.ascontiguousarray(y[:, m])
        assert x.shape == y.shape and np.array_equal(x.view(np.uint8), y.view(np.uint8)), (label, key)
    assert a["n_masked"] == b["n_masked"] and a["n_rays"] == b["n_rays"], label
    assert int(a["stats"][0]) == int(b["stats"][0]) and int(a["stats"][1]) == int(b["stats"][1]), label


def test_batch_equals_single_frames(sess):
    torch, dof = sess["torch"], sess["dof"]
    alone = render_alone(sess)
    frs, houts = make_frames(sess)
    b = dof.Batch(8, sess["params"], ray_records=True)
    b.set(batch_items(sess, frs, houts))
    b.run()
    got = [grab(torch, frs[k], houts[k]) for k in range(len(frs))]
    for k in range(len(frs)):
        same(got[k], alone[k], f"item {k}")
    nf, rays, visits, tests = b.totals()
    assert nf == len(frs) and rays == sum(a["n_rays"] for a in alone) and visits > 0 and tests > 0
    assert rays > 0


def test_batch_with_dilated_mask_equals_single_frames(sess):
    """Mask mode DOF_MASK_DILATE (an extra kernel between mask and
    compaction), batched vs alone."""
    torch, dof = sess["torch"], sess["dof"]
    params = sess["params"]
    try:
        sess["params"] = dataclasses.replace(params, mask_mode=synth.MASK_DILATE)
        alone = render_alone(sess)
        frs, houts = make_frames(sess)
        b = dof.Batch(4, sess["params"], ray_records=True)
        b.set(batch_items(sess, frs, houts))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone[k], f"dilated item {k}")
        base = render_alone(dict(sess, params=params))
        assert sum(a["n_rays"] for a in alone) > sum(a["n_rays"] for a in base)
    finally:
        sess["params"] = params


def test_batch_with_polygonal_gather_equals_single_frames(sess):
    """pp_polygon = 1: each item's gather kernel follows its own lens (the
    hexagonal item samples a hexagon, the others circles), batched vs alone."""
    torch, dof = sess["torch"], sess["dof"]
    params = sess["params"]
    try:
        sess["params"] = dataclasses.replace(params, pp_polygon=1)
        alone = render_alone(sess)
        frs, houts = make_frames(sess)
        b = dof.Batch(4, sess["params"], ray_records=True)
        b.set(batch_items(sess, frs, houts))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone[k], f"polygon item {k}")
        base = render_alone(dict(sess, params=params))
        assert not np.array_equal(alone[1]["gather"], base[1]["gather"])     # hexagonal lens: kernel changed
        assert np.array_equal(alone[0]["gather"], base[0]["gather"])         # circular lens: unchanged
    finally:
        sess["params"] = params


def test_batch_second_frame_with_history(sess):
    """Frame 1 of every session on frame 0's history (camera panned), batched
    vs alone."""
    torch, dof = sess["torch"], sess["dof"]
    f0 = render_alone(sess)
    hist = [torch.from_numpy(a["hist_out"]).cuda() for a in f0]
    prev = [it["cam"] for it in sess["items"]]
    moved = []
    for it in sess["items"]:
        c1 = dataclasses.replace(synth.pan_camera(it["cam"], 0.02), frame=1)
        moved.append(c1)
    saved = [it["cam"] for it in sess["items"]]
    try:
        for it, c1 in zip(sess["items"], moved):
            it["cam"] = c1
        alone = render_alone(sess, hist_in=hist, prev=prev)
        frs, houts = make_frames(sess)
        b = dof.Batch(4, sess["params"], ray_records=True)
        b.set(batch_items(sess, frs, houts, hist_in=hist, prev=prev))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone[k], f"frame 1 item {k}")
    finally:
        for it, c0 in zip(sess["items"], saved):
            it["cam"] = c0


def test_batch_with_taa_equals_single_frames(sess):
    """taa = 1 (one more full-resolution kernel after the composite): frame 0
    and then frame 1 on that TAA history, batched vs alone."""
    torch, dof = sess["torch"], sess["dof"]
    params = sess["params"]
    saved = [it["cam"] for it in sess["items"]]
    try:
        sess["params"] = dataclasses.replace(params, taa=1)
        alone0 = render_alone(sess)
        frs, houts = make_frames(sess)
        b = dof.Batch(4, sess["params"], ray_records=True)
        b.set(batch_items(sess, frs, houts))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone0[k], f"TAA frame 0 item {k}")
        hist = [torch.from_numpy(a["hist_out"]).cuda() for a in alone0]
        prev = list(saved)
        for it in sess["items"]:
            it["cam"] = dataclasses.replace(synth.pan_camera(it["cam"], 0.02), frame=1)
        alone1 = render_alone(sess, hist_in=hist, prev=prev)
        frs, houts = make_frames(sess)
        b.set(batch_items(sess, frs, houts, hist_in=hist, prev=prev))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone1[k], f"TAA frame 1 item {k}")
    finally:
        sess["params"] = params
        for it, c0 in zip(sess["items"], saved):
            it["cam"] = c0


def test_batch_with_all_taa_stages_and_jitter_equals_single_frames(sess):
    """taa = raster | post-filter | final on jittered cameras: frame 0 and
    then frame 1 on that history, batched vs alone (the raster stage hands
    the reduce and the composite its resolved colour per job)."""
    torch, dof = sess["torch"], sess["dof"]
    params = sess["params"]
    saved = [it["cam"] for it in sess["items"]]
    try:
        sess["params"] = dataclasses.replace(params, taa=synth.TAA_ALL)
        for k, it in enumerate(sess["items"]):
            it["cam"] = synth.jittered([it["cam"]], seed=synth.BASE_SEED + 40 + k)[0]
        alone0 = render_alone(sess)
        frs, houts = make_frames(sess)
        b = dof.Batch(4, sess["params"], ray_records=True)
        b.set(batch_items(sess, frs, houts))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone0[k], f"TAA all frame 0 item {k}")
        hist = [torch.from_numpy(a["hist_out"]).cuda() for a in alone0]
        prev = [it["cam"] for it in sess["items"]]
        for k, it in enumerate(sess["items"]):
            c1 = dataclasses.replace(synth.pan_camera(it["cam"], 0.02), frame=1)
            it["cam"] = synth.jittered([c1], seed=synth.BASE_SEED + 50 + k)[0]
        alone1 = render_alone(sess, hist_in=hist, prev=prev)
        frs, houts = make_frames(sess)
        b.set(batch_items(sess, frs, houts, hist_in=hist, prev=prev))
        b.run()
        for k in range(len(frs)):
            same(grab(torch, frs[k], houts[k]), alone1[k], f"TAA all frame 1 item {k}")
    finally:
        sess["params"] = params
        for it, c0 in zip(sess["items"], saved):
            it["cam"] = c0


def test_batch_item_matches_oracle(sess, orc):
    """The hexagonal-aperture item of a batch against the CPU oracle."""
    torch, dof = sess["torch"], sess["dof"]
    frs, houts = make_frames(sess)
    b = dof.Batch(4, sess["params"], ray_records=True)
    b.set(batch_items(sess, frs, houts))
    b.run()
    k = 1
    it = sess["items"][k]
    d = grab(torch, frs[k], houts[k])
    o = orc.render_frame(it["osc"], it["cam"], it["lens"], sess["params"], it["gb"])
    assert np.array_equal(d["mask"], o["mask"])
    assert np.array_equal(d["queue"], o["queue"]) and np.array_equal(d["ray_base"], o["ray_base"])
    assert np.array_equal(d["ray_hit"], o["ray_hit"])
    assert np.array_equal(d["ray_t"].view(np.uint32), o["ray_t"].view(np.uint32))
    np.testing.assert_allclose(d["recon"], o["recon"], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(d["hist_out"], o["hist_out"], rtol=1e-5, atol=1e-5)
    assert float(np.abs(d["colour"][..., :3] - o["colour"][..., :3]).max()) <= COLOUR_TOL


def test_batch_graph_replays(sess):
    """A captured batch run replayed three times, with eager work and a new
    item table (moved cameras) between replays; every replay equals the
    eager batch of the same table."""
    torch, dof = sess["torch"], sess["dof"]
    frs, houts = make_frames(sess)
    b = dof.Batch(4, sess["params"], ray_records=True)
    b.set(batch_items(sess, frs, houts))
    b.run()                       # warm-up outside the capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            b.run()
    torch.cuda.synchronize()
    saved = [it["cam"] for it in sess["items"]]
    try:
        for rep in range(3):
            for it, c0 in zip(sess["items"], saved):
                it["cam"] = dataclasses.replace(synth.pan_camera(c0, 0.01 * rep), frame=rep)
            ref_frs, ref_houts = make_frames(sess)
            ref = dof.Batch(4, sess["params"], ray_records=True)
            ref.set(batch_items(sess, ref_frs, ref_houts))
            ref.run()
            want = [grab(torch, ref_frs[k], ref_houts[k]) for k in range(len(ref_frs))]
            junk = torch.randn(1 << 20, device="cuda").sum()    # eager work between replays
            b.set(batch_items(sess, frs, houts))
            g.replay()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for k in range(len(frs)):
                same(grab(torch, frs[k], houts[k]), want[k], f"replay {rep} item {k}")
    finally:
        for it, c0 in zip(sess["items"], saved):
            it["cam"] = c0


def test_batch_rejects_bad_items(sess):
    torch, dof = sess["torch"], sess["dof"]
    frs, houts = make_frames(sess)
    items = batch_items(sess, frs, houts)
    b = dof.Batch(2, sess["params"], ray_records=True)
    with pytest.raises(dof.DofError) as e:
        b.set(items[:3])
    assert e.value.code == dof.DOF_E_NOMEM
    dup = [items[0], items[0]]
    with pytest.raises(dof.DofError) as e:
        b.set(dup)
    assert e.value.code == dof.DOF_E_INVALID
    items[1].scratch_bytes -= 256
    with pytest.raises(dof.DofError) as e:
        b.set(items[:2])
    assert e.value.code == dof.DOF_E_NOMEM and "item 1" in str(e.value)
