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
