"""Autotuning of the pass's launch shapes (none of them changes a result).

Searched per workload, by HIP-event time of the same sample of frames:

* trace_blocks -- the persistent traversal's grid: too few blocks leave
  compute units idle while long rays drain, too many only add waves that
  find no work (multiples of the compute-unit count, and the library default
  of as many blocks as fit at once);
* trace_stack -- LDS stack entries per traversal lane (16, 24, 32): fewer
  entries leave room for more resident blocks, more make stack overflows
  (recovered through parent links) rarer;
* trace_grab -- rays a wave takes from the traversal's work counters at a
  time (its queue width; 32 to 256);
* trace_refill -- idle lanes at which a wave takes new rays;
* trace_leaf_batch -- lanes with a pending leaf at which a wave runs its
  triangle tests;
* gather_window -- the LDS window of the post-process gather's staged tiles
  (32, 40, 48 texels, or -1: every tap from global memory);
* trace_order -- rays handed out from the end of the queue (2: bottom image
  rows first) or from its start (1); the last rays handed out set the
  persistent grid's tail;
* trace_steps -- node visits per lane in one iteration of the traversal
  loop (3, 4): more visits between the loop's refill and triangle-test
  decisions save their ballots but hold finished lanes longer.

The search is coordinate descent from the library defaults: one knob at a
time over its candidates with the others held, keeping the fastest unless the
value already held is within `margin` (1 %) of it -- differences that small
are run-to-run noise, and chasing them only makes the pick flip between runs.
"""

from __future__ import annotations

KNOB_SPACE = {
    "trace_blocks": None,                      # filled from the device (candidate_blocks)
    "trace_stack": (16, 24, 32),
    "trace_grab": (32, 64, 128, 256),
    "trace_refill": (8, 16, 24),
    "trace_leaf_batch": (16, 24, 32, 40),
    "gather_window": (-1, 32, 40, 48),
    "trace_order": (2, 1),
    "trace_steps": (4, 3),
}
DEFAULTS = {"trace_blocks": 0, "trace_stack": 24, "trace_grab": 64, "trace_refill": 16, "trace_leaf_batch": 32,
            "gather_window": -1, "trace_order": 2, "trace_steps": 4}


def candidate_blocks(extra=()):
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return sorted({0, *(cus * k for k in (4, 6, 7, 8, 9, 10, 12)), *extra})


def pick(times, incumbent=None, margin: float = 0.0):
    """The fastest candidate of {candidate: ms}, or the incumbent when it is
    within a relative margin of the fastest."""
    best = min(times, key=times.get)
    if incumbent in times and times[incumbent] <= times[best] * (1.0 + margin):
        return incumbent
    return best


def tune(run, candidates, reps: int = 3, incumbent=None, margin: float = 0.0):
    """run(candidate) renders a fixed sample of work (same every call);
    returns (best candidate, {candidate: median ms})."""
    import statistics

    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = {}
    for c in candidates:
        run(c)                     # warm-up for this candidate
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            e0.record()
            run(c)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        times[c] = statistics.median(ms)
    return pick(times, incumbent, margin), times


def search(run, space=None, reps: int = 2, order=None, margin: float = 0.01):
    """Coordinate descent over the knobs: run(config) renders the sample with
    config (a dict with every knob of `space`).  Returns (best config,
    {knob: {value: ms}})."""
    space = dict(KNOB_SPACE if space is None else space)
    if space.get("trace_blocks", ()) is None:
        space["trace_blocks"] = candidate_blocks()
    cfg = {k: DEFAULTS[k] for k in space}
    table = {}
    for knob in order or list(space):
        best, times = tune(lambda v: run({**cfg, knob: v}), space[knob], reps=reps, incumbent=cfg[knob],
                           margin=margin)
        cfg[knob] = best
        table[knob] = times
    return cfg, table


def split(cfg):
    """(trace_blocks, the dof_params knobs) of a configuration."""
    cfg = dict(cfg)
    return cfg.pop("trace_blocks", 0), cfg
