"""The traversal-grid autotuner: every candidate is timed, the fastest is
returned, and the grid never changes the result (the traversal is exact for
any number of persistent blocks)."""

import numpy as np
import pytest

from paper_2210_06158_amd import synth

pytestmark = pytest.mark.gpu


def test_tuner_times_every_candidate_and_grids_agree():
    import torch
    from paper_2210_06158_amd import dof, tune
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    gs = dof.Scene(scene)
    gs.build_bvh()
    gb = gs.render_gbuffer(cam, lens)
    frames, outs = {}, {}

    def run(tb):
        if tb not in frames:
            frames[tb] = dof.Frame(cam.width, cam.height, params, trace_blocks=tb)
        frames[tb].render(gs, cam, lens, gb, None, dof.history_alloc(cam.width, cam.height))

    cands = [0, 64, 256, 1024]
    best, times = tune.tune(run, cands, reps=2)
    assert set(times) == set(cands) and best in cands
    assert times[best] == min(times.values()) and all(t > 0 for t in times.values())
    torch.cuda.synchronize()
    ref = frames[0].colour.cpu().numpy()
    for tb in cands[1:]:
        assert np.array_equal(frames[tb].colour.cpu().numpy(), ref), tb
        assert np.array_equal(frames[tb].mask.cpu().numpy(), frames[0].mask.cpu().numpy()), tb


def test_extreme_grids_agree():
    """One block (two waves take every pool of rays in turn), three blocks,
    and the largest grid (most waves find no work): frames and a batch of
    two sessions equal the default grid's, bit for bit."""
    import dataclasses
    import torch
    from paper_2210_06158_amd import dof
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    gs = dof.Scene(scene)
    gs.build_bvh()
    gb = gs.render_gbuffer(cam, lens)
    cam2 = dataclasses.replace(cam, width=130, height=66)
    gb2 = gs.render_gbuffer(cam2, lens)
    out = {}
    for tb in (0, 1, 3, 4096):
        fr = dof.Frame(cam.width, cam.height, params, trace_blocks=tb)
        fr.render(gs, cam, lens, gb, None, dof.history_alloc(cam.width, cam.height))
        frs = [dof.Frame(c.width, c.height, params) for c in (cam, cam2)]
        hs = [dof.history_alloc(c.width, c.height) for c in (cam, cam2)]
        b = dof.Batch(2, params, trace_blocks=tb)
        b.set([frs[0].item(gs, cam, lens, gb, None, hs[0]), frs[1].item(gs, cam2, lens, gb2, None, hs[1])])
        b.run()
        torch.cuda.synchronize()
        out[tb] = [fr.colour.cpu().numpy(), fr.stats.cpu().numpy()[:2]] + [f.colour.cpu().numpy() for f in frs]
    assert out[0][1][1] > 1000                      # rays in the frame
    for tb in (1, 3, 4096):
        for a, r in zip(out[tb], out[0]):
            assert np.array_equal(a, r), tb


def test_launch_knobs_never_change_a_result():
    """Every value of every launch knob the autotuner searches (traversal
    stack depth, queue width, refill and leaf-batch thresholds, hand-out
    order, node visits per loop iteration, the gather's LDS window, including
    no staging) renders the same frame bit for bit --
    colour, mask, history -- on the 256 x 256 workload and a second frame
    with history, alone and in a batch of two."""
    import dataclasses
    import torch
    from paper_2210_06158_amd import dof, tune
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    gs = dof.Scene(scene)
    gs.build_bvh()
    cam1 = synth.pan_camera(dataclasses.replace(cam, frame=1), 0.02)
    gbs = [gs.render_gbuffer(c, lens) for c in (cam, cam1)]

    def render(knobs, tb=0):
        fr = dof.Frame(cam.width, cam.height, params, trace_blocks=tb, knobs=knobs)
        h0, h1 = dof.history_alloc(cam.width, cam.height), dof.history_alloc(cam.width, cam.height)
        fr.render(gs, cam, lens, gbs[0], None, h0)
        fr.render(gs, cam1, lens, gbs[1], h0, h1, prev_cam=cam, prev_lens=lens)
        frs = [dof.Frame(cam.width, cam.height, params, knobs=knobs) for _ in range(2)]
        hs = [dof.history_alloc(cam.width, cam.height) for _ in range(2)]
        b = dof.Batch(2, params, trace_blocks=tb, knobs=knobs)
        b.set([frs[0].item(gs, cam, lens, gbs[0], None, hs[0]),
               frs[1].item(gs, cam1, lens, gbs[1], h0, hs[1], prev_cam=cam, prev_lens=lens)])
        b.run()
        torch.cuda.synchronize()
        return [fr.colour.cpu().numpy(), fr.mask.cpu().numpy(), h1.cpu().numpy(), fr.stats.cpu().numpy()[:2],
                frs[0].colour.cpu().numpy(), frs[1].colour.cpu().numpy(), hs[1].cpu().numpy()]

    ref = render({})
    assert ref[3][1] > 1000
    cases = [{k: v} for k, vals in tune.KNOB_SPACE.items() if k != "trace_blocks" for v in vals]
    cases.append({"trace_stack": 16, "trace_grab": 1, "trace_refill": 1, "trace_leaf_batch": 1, "gather_window": 32,
                  "trace_steps": 4})
    cases.append({"trace_stack": 32, "trace_grab": 256, "trace_refill": 64, "trace_leaf_batch": 64,
                  "gather_window": -1, "trace_steps": 3})
    for knobs in cases:
        got = render(knobs)
        for a, r in zip(got, ref):
            assert np.array_equal(a, r), knobs


def test_search_picks_the_fastest_per_knob():
    """Coordinate descent: each knob's candidates are all timed with the
    others held at the running best, and the fastest is kept (no margin)."""
    import torch
    from paper_2210_06158_amd import dof, tune
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    gs = dof.Scene(scene)
    gs.build_bvh()
    gb = gs.render_gbuffer(cam, lens)
    h = dof.history_alloc(cam.width, cam.height)
    seen = []

    def run(cfg):
        seen.append(dict(cfg))
        tb, knobs = tune.split(cfg)
        dof.Frame(cam.width, cam.height, params, trace_blocks=tb, knobs=knobs).render(gs, cam, lens, gb, None, h)

    space = {"trace_blocks": (0, 256), "trace_stack": (16, 24), "gather_window": (-1, 48)}
    cfg, table = tune.search(run, space=space, reps=1, margin=0.0)
    assert set(table) == set(space)
    for k, times in table.items():
        assert set(times) == set(space[k]) and cfg[k] == min(times, key=times.get)
    assert all(set(c) == set(space) for c in seen)


def test_traversal_statistics_add_up_over_the_counter_slots():
    """With triangle tests run whenever any lane has a pending leaf
    (trace_leaf_batch 1), each ray's node visits, triangle tests and stack
    drops follow from that ray alone, so a frame's totals do not depend on
    the persistent grid.  One block (every wave adds into one statistics
    slot), 16 blocks (two per slot) and the default grid give the same
    totals, and a batch of the frame twice gives twice them: the slots are
    summed completely, once."""
    import torch
    from paper_2210_06158_amd import dof
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    gs = dof.Scene(scene)
    gs.build_bvh()
    gb = gs.render_gbuffer(cam, lens)
    knobs = {"trace_leaf_batch": 1, "trace_stack": 16}

    def frame_totals(tb):
        fr = dof.Frame(cam.width, cam.height, params, trace_blocks=tb, knobs=knobs)
        fr.render(gs, cam, lens, gb, None, dof.history_alloc(cam.width, cam.height))
        torch.cuda.synchronize()
        s = fr.stats.cpu().numpy()
        s64 = s.view(np.int64)
        return int(s[1]), int(s64[1]), int(s64[2]), int(s[6])

    one = frame_totals(1)
    rays, visits, tests, drops = one
    assert rays > 1000 and visits >= rays and 0 < tests <= 2 * visits
    assert frame_totals(16) == one and frame_totals(0) == one

    frs = [dof.Frame(cam.width, cam.height, params, knobs=knobs) for _ in range(2)]
    b = dof.Batch(2, params, trace_blocks=16, knobs=knobs)
    hs = [dof.history_alloc(cam.width, cam.height) for _ in range(2)]   # kept alive: the items hold pointers
    b.set([f.item(gs, cam, lens, gb, None, h) for f, h in zip(frs, hs)])
    b.run()
    torch.cuda.synchronize()
    nf, brays, bvisits, btests = b.totals()
    assert nf == 2 and (brays, bvisits, btests) == (2 * rays, 2 * visits, 2 * tests)
