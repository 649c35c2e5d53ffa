"""Autotuning of the launch parameters that are runtime choices.

The persistent traversal's grid (dof_params.trace_blocks) is the one launch
parameter the library leaves to its caller: too few blocks leave compute
units idle while long rays drain, too many only add waves that find no work.
The tuner renders the same frames with each candidate grid (multiples of the
compute-unit count, plus the library default of as many blocks as fit at
once) and keeps the fastest by HIP-event time.  Tile size (16) and stack
depth are compile-time constants of the kernels.
"""

from __future__ import annotations


def candidate_blocks(extra=()):
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return sorted({0, *(cus * k for k in (4, 6, 7, 8, 9, 10, 12)), *extra})


def tune(run, candidates, reps: int = 3):
    """run(trace_blocks) renders a fixed sample of work (same every call);
    returns (best candidate, {candidate: median ms})."""
    import statistics

    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = {}
    for c in candidates:
        run(c)                     # warm-up for this grid
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            e0.record()
            run(c)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        times[c] = statistics.median(ms)
    best = min(times, key=times.get)
    return best, times
