"""Serving loop: continuous batching of Poisson frame requests over resident
sessions.  Every served frame must equal the same frame rendered alone (bit
for bit: a session's result depends only on its own frame sequence), every
request is either served or superseded by a newer one of its session, and
sessions are admitted only while they fit the HBM budget."""

import pytest

from paper_2210_06158_amd import synth

pytestmark = pytest.mark.gpu

SIZES = ((256, 144), (320, 180), (192, 108))


@pytest.fixture(scope="module")
def server():
    import torch
    from paper_2210_06158_amd import serve
    torch.cuda.set_device(0)
    params = synth.Params(m=4)
    specs = serve.serving_specs(6, seed=synth.BASE_SEED + 7000, tri_lo=2e3, tri_hi=2e4, sizes=SIZES)
    srv = serve.Server(64 << 30, params, max_batch=4, max_inflight=2, ring=3)
    for sp in specs:
        assert srv.admit(sp)
    torch.cuda.synchronize()
    return dict(torch=torch, serve=serve, srv=srv, specs=specs, params=params)


@pytest.mark.parametrize("mode", ["batched", "single"])
def test_every_served_frame_equals_the_frame_alone(server, mode):
    torch, serve, srv = server["torch"], server["serve"], server["srv"]
    arrivals = serve.poisson_arrivals(len(srv.sessions), 120.0, 0.4, seed=11)
    kept = {}
    m = srv.run(arrivals, 0.4, mode=mode, keep=kept)
    assert m["offered"] == len(arrivals) and m["served"] + m["superseded"] == m["offered"]
    assert m["served"] > 0 and m["p50_latency_ms"] > 0 and m["p99_latency_ms"] >= m["p50_latency_ms"]
    if mode == "batched":
        assert m["mean_batch"] >= 1.0
    else:
        assert m["mean_batch"] == 1.0
    for sid, frames in kept.items():
        scene, cams, lens, _ = synth.scene_session(server["specs"][sid])
        alone = serve.RingSession(scene, cams, lens, server["params"], ring=3)
        for k, got in enumerate(frames):
            alone.prepare(k)
            alone.render()
            torch.cuda.synchronize()
            assert torch.equal(alone.frame.colour, got), (mode, sid, k)


def test_admission_by_memory_budget(server):
    serve, srv = server["serve"], server["srv"]
    small = serve.Server(srv.sessions[0].bytes + (1 << 20), server["params"], max_batch=2, ring=3)
    assert small.admit(server["specs"][0])
    assert not small.admit(server["specs"][1])
    assert small.rejected == 1 and len(small.sessions) == 1 and small.used <= small.budget


def test_served_frames_match_the_oracle(server, orc):
    """The first two frames served for two sessions (continuous batching,
    FP16 G-buffer and output) against the CPU oracle rendering the same views
    in sequence, the second on the first's history, from the same G-buffers
    (the oracle's, rounded to FP16 as the sessions store them): colour within
    1e-3 and the history record after the second frame within 1e-5."""
    import numpy as np
    torch, serve, srv = server["torch"], server["serve"], server["srv"]
    arrivals = [(0.0, 0), (0.0, 1), (0.05, 0), (0.05, 1)]
    kept = {}
    m = srv.run(arrivals, 0.1, mode="batched", keep=kept)
    assert m["served"] == 4 and m["superseded"] == 0
    for sid in (0, 1):
        sess = srv.sessions[sid]
        scene, cams, lens, _ = synth.scene_session(server["specs"][sid])
        osc = orc.OracleScene(scene)
        osc.build_bvh()
        hist, prev = None, None
        for k in range(2):
            cam = sess.cam(k)
            g = orc.gbuffer(osc, sess.cams[k % len(sess.ring)], lens)
            gb = orc.GBuffer(g.colour.astype(np.float16).astype(np.float32), g.depth,
                             g.normal.astype(np.float16).astype(np.float32))
            o = orc.render_frame(osc, cam, lens, server["params"], gb, hist_in=hist, prev_cam=prev,
                                 prev_lens=lens if prev is not None else None, debug=False)
            got = kept[sid][k].float().cpu().numpy()
            err = float(np.abs(got[..., :3] - o["colour"][..., :3]).max())
            assert err <= 1e-3, (sid, k, err)
            hist, prev = o["hist_out"], cam
        # the session's history after its second frame equals the oracle's
        np.testing.assert_allclose(sess.history_out().cpu().numpy(), hist, rtol=1e-5, atol=1e-5)
