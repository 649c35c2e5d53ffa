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
