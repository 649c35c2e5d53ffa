"""dof_render_frame_noalloc (the library's own scratch buffer, for callers
that cannot allocate) against dof_render_frame with a caller buffer: two
calls in a row, the second on a smaller frame with history, bit for bit."""

import dataclasses

import numpy as np
import pytest

from paper_2210_06158_amd import synth

pytestmark = pytest.mark.gpu


def _gpu(torch, gb):
    return (torch.from_numpy(gb.colour).cuda(), torch.from_numpy(gb.depth).cuda(), torch.from_numpy(gb.normal).cuda())


def test_noalloc_equals_render_frame_on_two_calls(orc):
    import torch
    from paper_2210_06158_amd import dof
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    osc = orc.OracleScene(scene)
    osc.build_bvh()
    gs = dof.Scene(scene)
    gs.build_bvh()
    cams = [cam, dataclasses.replace(synth.pan_camera(cam, 0.02), width=128, height=96, frame=1)]
    hist_in = [None, None]
    for call, c in enumerate(cams):
        print(f"noalloc call {call}: {c.width}x{c.height}", flush=True)
        g = _gpu(torch, orc.gbuffer(osc, c, lens))
        if call == 1:
            # history of the smaller frame: a frame of its own size rendered the ordinary way
            h0 = dof.history_alloc(c.width, c.height)
            dof.Frame(c.width, c.height, params).render(gs, c, lens, g, None, h0)
            hist_in[1] = h0
        pc = c if call == 1 else None
        ref = dof.Frame(c.width, c.height, params)
        ref_h = dof.history_alloc(c.width, c.height)
        ref.render(gs, c, lens, g, hist_in[call], ref_h, prev_cam=pc, prev_lens=lens)
        na = dof.Frame(c.width, c.height, params)
        na_h = dof.history_alloc(c.width, c.height)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        na.render_noalloc(gs, c, lens, g, hist_in[call], na_h, prev_cam=pc, prev_lens=lens)
        torch.cuda.synchronize()
        if call == 1:
            assert torch.cuda.mem_get_info()[0] == free0          # nothing allocated on the device
        assert torch.equal(na.colour, ref.colour), call
        assert torch.equal(na.mask, ref.mask), call
        assert torch.equal(na_h, ref_h), call
        assert torch.equal(na.stats, ref.stats), call
        assert int(na.stats[1]) > 0
        # and against the oracle's mask (the pass's integer decisions)
        o = orc.render_frame(osc, c, lens, params, orc.gbuffer(osc, c, lens),
                             hist_in=hist_in[call].cpu().numpy() if hist_in[call] is not None else None,
                             prev_cam=pc, prev_lens=lens if pc is not None else None, debug=False)
        assert np.array_equal(na.mask.cpu().numpy(), o["mask"]), call
