"""Resident sessions: what one viewer of the hybrid depth-of-field pass keeps in
HBM between frames -- its scene and BVH, a G-buffer slot, two history records
(ping-pong) and the buffers of its frame (scratch, colour, mask, stats).

A session renders frame k of its camera path either alone (dof_render_frame)
or as one item of a batch (dof_batch_*).  Either way the result depends only
on the session's own earlier frames, so a frame is identical alone and in a
mix.  Every device byte a session holds comes from the library's size
queries, which is what admission by memory budget counts.
"""

from __future__ import annotations

import dataclasses

from . import dof, synth


def resident_bytes(scene_arena_bytes: int, width: int, height: int, params) -> int:
    """HBM a session holds: scene arena, one FP16 G-buffer, two history
    records, frame scratch, FP16 colour, mask and stats."""
    px = width * height
    return (scene_arena_bytes + px * 20 + 2 * dof.history_bytes(width, height)
            + dof.scratch_bytes(width, height, params) + px * 8 + px // 4 + 32)


class Session:
    def __init__(self, scene, cams, lens, params, device="cuda"):
        import torch
        self.cams, self.lens, self.params = cams, lens, params
        self.W, self.H = cams[0].width, cams[0].height
        self.ntri = scene.ntri
        self.gs = dof.Scene(scene, device=device)
        self.gs.build_bvh()
        px = self.W * self.H
        self.gb = (torch.empty((self.H, self.W, 4), dtype=torch.float16, device=device),
                   torch.empty((self.H, self.W), dtype=torch.float32, device=device),
                   torch.empty((self.H, self.W, 4), dtype=torch.float16, device=device))
        self.hist = [dof.history_alloc(self.W, self.H, device=device), dof.history_alloc(self.W, self.H, device=device)]
        self.frame = dof.Frame(self.W, self.H, params, out_format=dof.RGBA16F, device=device)
        self.done = 0              # frames rendered so far (history chain position)
        self.gb_frame = -1
        self.bytes = resident_bytes(self.gs.arena.numel(), self.W, self.H, params)
        assert px > 0

    @classmethod
    def from_spec(cls, spec, m=8, device="cuda", leaf_split=None):
        scene, cams, lens, params = synth.scene_session(spec)
        params.m = m
        if leaf_split is not None:
            scene = dataclasses.replace(scene, leaf_split=leaf_split)
        return cls(scene, cams, lens, params, device=device)

    def cam(self, k):
        c = self.cams[k % len(self.cams)]
        return c if c.frame == k else dataclasses.replace(c, frame=k)

    def prepare(self, k):
        """Render the G-buffer of path frame k into the session's slot (the
        input a client would upload; not part of the pass)."""
        if self.gb_frame != k:
            self.gs.render_gbuffer_into(self.cam(k), self.lens, *self.gb)
            self.gb_frame = k

    def _args(self):
        k = self.done
        prev = self.cam(k - 1) if k > 0 else None
        hin = self.hist[(k + 1) % 2] if prev is not None else None
        return k, prev, hin, self.hist[k % 2]

    def item(self):
        """Batch item of the next frame (call prepare(next_index) first)."""
        k, prev, hin, hout = self._args()
        return self.frame.item(self.gs, self.cam(k), self.lens, self.gb, hin, hout, prev_cam=prev,
                               prev_lens=self.lens)

    def render(self):
        """Render the next frame alone."""
        k, prev, hin, hout = self._args()
        self.frame.render(self.gs, self.cam(k), self.lens, self.gb, hin, hout, prev_cam=prev, prev_lens=self.lens)
        self.done += 1

    def advance(self):
        """Mark the next frame as rendered (after it ran inside a batch)."""
        self.done += 1

    def history_out(self):
        return self.hist[(self.done - 1) % 2]
