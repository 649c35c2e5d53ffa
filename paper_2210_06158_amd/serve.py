"""Serving loop: continuous batching of frame requests from many sessions.

Sessions (scene + BVH, history, frame buffers and a ring of G-buffers) stay
resident in HBM; a session is admitted only while the sum of the sessions'
resident bytes fits the HBM budget.  Frame requests arrive per session as a
Poisson process.  A session has at most one frame on the GPU (its history
chains frames), and a request that arrives while an older request of the same
session is still waiting replaces it (the newest view wins, as in real-time
rendering; the replaced request is counted as superseded).

Batched mode: whenever fewer than `max_inflight` batches are on the GPU, every
waiting session whose previous frame has finished joins the next batch
(up to `max_batch`), which is launched on the next of `max_inflight` streams
-- requests that arrive while other frames run are admitted as soon as their
session is free, and consecutive batches overlap on the device.  Single mode
serves the same requests one frame at a time (one dof_render_frame each).

Latency of a frame = completion - arrival, where completion is read from an
event recorded after the frame's work, on the device clock aligned to the host
clock at the start of the run.
"""

from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import dof, sessions, synth

SESSION_SIZES_SERVING = ((1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))


def serving_specs(n: int, seed: int = synth.BASE_SEED + 6000, tri_lo: float = 0.2e6, tri_hi: float = 1.0e6,
                  sizes=SESSION_SIZES_SERVING) -> list:
    """n sessions, resolution uniform over `sizes`, triangle budget uniform in
    [tri_lo, tri_hi] (same scene recipe as the 1080p workload)."""
    rng = synth.SplitMix64(seed)
    cls = rng.uniform(n)
    tri = rng.uniform(n, tri_lo, tri_hi)
    out = []
    for i in range(n):
        w, h = sizes[min(int(cls[i] * len(sizes)), len(sizes) - 1)]
        scale = tri[i] / 1183042.0
        out.append((seed + 1 + i, w, h, max(1, int(round(4096 * scale))), max(1, int(round(50000 * scale)))))
    return out


def poisson_arrivals(n_sessions: int, rate_hz: float, duration_s: float, seed: int) -> list:
    """Sorted (time, session) arrivals: exponential gaps of mean 1/rate per
    session, from a seeded SplitMix64 stream."""
    rng = synth.SplitMix64(seed)
    out = []
    for sid in range(n_sessions):
        t = 0.0
        while True:
            u = float(rng.uniform(1)[0])
            t += -math.log(1.0 - u) / rate_hz
            if t >= duration_s:
                break
            out.append((t, sid))
    out.sort()
    return out


class RingSession(sessions.Session):
    """A session whose client G-buffers are resident: a ring of `ring`
    pre-rendered views of its camera path, frame k using view k mod ring."""

    def __init__(self, scene, cams, lens, params, ring=4, device="cuda"):
        import torch
        super().__init__(scene, cams[:ring], lens, params, device=device)
        self.ring = [self.gb]
        for _ in range(ring - 1):
            self.ring.append(tuple(torch.empty_like(t) for t in self.gb))
        for k in range(ring):
            self.gs.render_gbuffer_into(self.cams[k], self.lens, *self.ring[k])
        self.bytes += (ring - 1) * self.W * self.H * 20

    def prepare(self, k):
        self.gb = self.ring[k % len(self.ring)]
        self.gb_frame = k


class Server:
    def __init__(self, budget_bytes: int, params, max_batch: int = 32, max_inflight: int = 2, ring: int = 4,
                 device="cuda", leaf_split=None):
        import torch
        self.torch = torch
        self.budget = budget_bytes
        self.leaf_split = leaf_split      # BVH leaf split level of the sessions' scenes (None: the scene's own)
        self.params = params
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.ring = ring
        self.device = device
        self.sessions = []
        self.used = 0
        self.rejected = 0
        self.streams = [torch.cuda.Stream() for _ in range(max_inflight)]
        self.batches = [dof.Batch(max_batch, params, device=device) for _ in range(max_inflight)]

    def admit(self, spec) -> bool:
        """Create a resident session if its bytes fit the budget."""
        _, w, h, ns, nb = spec
        scene, cams, lens, _ = synth.scene_session(spec)
        if self.leaf_split is not None:
            scene = dataclasses.replace(scene, leaf_split=self.leaf_split)
        need = sessions.resident_bytes(dof.scene_bytes_for(scene), w, h, self.params) + (self.ring - 1) * w * h * 20
        if self.used + need > self.budget:
            self.rejected += 1
            return False
        s = RingSession(scene, cams, lens, self.params, ring=self.ring, device=self.device)
        self.sessions.append(s)
        self.used += s.bytes
        return True

    def reset(self):
        for s in self.sessions:
            s.done = 0

    def run(self, arrivals, duration_s: float, mode: str = "batched", keep=None, max_batch=None,
            max_inflight=None):
        """Serve `arrivals` ((t, session) sorted, t in seconds from the start)
        in real time.  keep (optional dict) receives, per session, clones of
        the colour of every served frame.  max_batch / max_inflight override
        the server's limits for this run.  Returns a metrics dict."""
        torch = self.torch
        assert mode in ("batched", "single")
        max_batch = self.max_batch if max_batch is None else min(max_batch, self.max_batch)
        max_inflight = self.max_inflight if max_inflight is None else min(max_inflight, self.max_inflight)
        nsess = len(self.sessions)
        self.reset()
        pending = {}                    # session -> arrival time of its newest waiting request
        busy = [False] * nsess
        inflight = []                   # (end event, [(session, arrival)], stream index)
        lat, served, superseded, batch_sizes = [], 0, 0, []
        next_stream = 0
        ai = 0
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ref.record(self.streams[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def retire():
            """Retire finished batches, oldest first."""
            nonlocal served
            while inflight and inflight[0][0].query():
                ev, frames, _ = inflight.pop(0)
                done_t = ref.elapsed_time(ev) * 1e-3
                for sid, at in frames:
                    lat.append(done_t - at)
                    busy[sid] = False
                    served += 1
                    if keep is not None:
                        keep.setdefault(sid, []).append(self.sessions[sid].frame.colour.clone())

        while True:
            now = time.perf_counter() - t0
            while ai < len(arrivals) and arrivals[ai][0] <= now:
                t, sid = arrivals[ai]
                if sid < nsess:
                    if sid in pending:
                        superseded += 1
                    pending[sid] = t
                ai += 1
            retire()
            if ai >= len(arrivals) and not pending and not inflight:
                break
            ready = [sid for sid in sorted(pending, key=pending.get) if not busy[sid]]
            if ready and len(inflight) < max_inflight:
                take = ready[:max_batch] if mode == "batched" else ready[:1]
                si = next_stream
                next_stream = (next_stream + 1) % max_inflight
                st = self.streams[si]
                with torch.cuda.stream(st):
                    frames = []
                    for sid in take:
                        s = self.sessions[sid]
                        s.prepare(s.done)
                        frames.append((sid, pending.pop(sid)))
                        busy[sid] = True
                    if mode == "batched":
                        b = self.batches[si]
                        b.set([self.sessions[sid].item() for sid, _ in frames])
                        b.run()
                        for sid, _ in frames:
                            self.sessions[sid].advance()
                    else:
                        self.sessions[frames[0][0]].render()
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(st)
                inflight.append((ev, frames, si))
                batch_sizes.append(len(frames))
                continue
            # nothing to launch now: wait briefly for the GPU or the next arrival
            wait = 2e-4
            if ai < len(arrivals):
                wait = min(wait, max(arrivals[ai][0] - (time.perf_counter() - t0), 0.0))
            if wait > 0:
                time.sleep(wait)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1e3
        offered = sum(1 for t, sid in arrivals if sid < nsess)
        return {
            "mode": mode,
            "max_batch": max_batch if mode == "batched" else 1,
            "max_inflight": max_inflight,
            "offered": offered,
            "served": served,
            "superseded": superseded,
            "frames_per_s": round(served / wall, 2),
            "wall_s": round(wall, 3),
            "p50_latency_ms": round(float(np.percentile(lat_ms, 50)), 3) if served else None,
            "p99_latency_ms": round(float(np.percentile(lat_ms, 99)), 3) if served else None,
            "mean_batch": round(float(np.mean(batch_sizes)), 2) if batch_sizes else 0.0,
            "launches": len(batch_sizes),
        }
