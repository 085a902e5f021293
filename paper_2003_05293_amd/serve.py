"""Request loop of the serving form: replays timed hologram requests through
the continuous-batching engine (hg_engine_*) in real time.

Each request is submitted when its arrival time comes; the loop then keeps
stepping the engine (every step advances all admitted holograms by one
iteration in one launch) and polls for completions.  Latency is measured on
the host clock from arrival to the moment the loop observes the finished
hologram.  Output buffers come from a small pool of GPU tensors and return
to it when their request completes.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Sequence

from . import Engine


@dataclasses.dataclass
class ServeResult:
    latencies_s: List[float]
    wall_s: float
    completed: int
    steps: int

    def percentile(self, q: float) -> float:
        import numpy as np
        return float(np.percentile(np.asarray(self.latencies_s), q)) if self.latencies_s else 0.0


def replay(requests: Sequence, optics, engine: Engine, stream=None, max_pixels: int = None,
           on_done=None) -> ServeResult:
    """requests: objects with .arrival_s (seconds from the start) and .job
    (grid, spots, iterations, compression, seed), sorted by arrival.
    on_done(request, phi) is called for each completed request before its
    output buffer is reused."""
    import torch
    if max_pixels is None:
        max_pixels = max(r.job.grid.W * r.job.grid.H for r in requests)
    free = []
    pending = collections.deque(requests)
    inflight = {}
    lat = []
    steps = 0
    t0 = time.perf_counter()
    while pending or inflight:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival_s <= now:
            r = pending.popleft()
            buf = free.pop() if free else torch.empty(max_pixels, dtype=torch.float32,
                                                     device="cuda")
            j = r.job
            t = engine.submit(j.grid, optics, j.spots, j.iterations, j.compression, j.seed, buf)
            inflight[t] = (r, buf)
        if inflight:
            engine.step(stream)
            steps += 1
            done = [t for t in list(inflight) if engine.poll(t)]
            if done:
                t_obs = time.perf_counter() - t0
                for t in done:
                    r, buf = inflight.pop(t)
                    lat.append(t_obs - r.arrival_s)
                    if on_done is not None:
                        on_done(r, buf[: r.job.grid.W * r.job.grid.H])
                    free.append(buf)
        elif pending:
            time.sleep(max(0.0, pending[0].arrival_s - (time.perf_counter() - t0)))
    return ServeResult(lat, time.perf_counter() - t0, len(lat), steps)
