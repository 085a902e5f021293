"""Autotuner of the pass launch parameters (hg_tune).

A pass runs on min(tiles, cap) blocks that take its tiles of pixels
dynamically; the caps of the compressed and of the full-grid per-pixel
passes, the form of the compressed pass (two sincos per pixel-spot pair, or
one shared complex exponential) and, for one hologram at a time, whether
its compressed passes run chained in one launch are the tunable parameters.
Partial sums are kept per tile, so the caps never change the results; the
form changes the rounding only.

For a workload -- one hologram shape, or a whole batch of jobs -- the tuner
times every candidate on the GPU (HIP events on the launch stream, after a
warm-up run) and keeps the fastest.  Results are cached in a JSON table
keyed by the workload's shape:

    table = autotune.Table(path)            # loads the file if it exists
    tune = table.single(grid, optics, spots, 30, 1/16)   # tunes on a miss
    phi = hg.cswgs(grid, optics, spots, 30, 1/16, seed, tune=tune)
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional

SUBSET_CAPS = (256, 512, 768, 1024, 1536, 2048, 4096)
FULL_CAPS = (1024, 2048, 4096)
PASS_FORMS = (0, 1)
LAUNCHES = (0, 1)  # chain_passes: chained compressed passes (single hologram) or not


def _hg():
    import paper_2003_05293_amd as hg
    return hg


def single_key(grid, n: int, iterations: int, compression: float, precision: str) -> str:
    return f"single:{precision}:{grid.W}x{grid.H}:n{n}:i{iterations}:c{compression:.6g}"


def batch_key(jobs) -> str:
    """Shape of a batch: the sorted multiset of its jobs' shapes."""
    shapes = sorted(f"{j.grid.W}x{j.grid.H}:n{int(j.spots_dev.shape[1])}:i{j.iterations}:"
                    f"c{j.compression:.6g}:f{j.flags & 0xff}" for j in jobs)
    digest = hashlib.sha1("|".join(shapes).encode()).hexdigest()[:16]
    return f"batch:{len(jobs)}:{digest}"


def _time(run, reps: int, stream) -> float:
    """Mean milliseconds of run() over reps calls, after one warm-up call."""
    import torch
    run()
    stream.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        run()
    b.record(stream)
    stream.synchronize()
    return a.elapsed_time(b) / reps


def _candidates(subset_caps: Iterable[int], full_caps: Iterable[int],
                forms: Iterable[int] = PASS_FORMS,
                launches: Iterable[int] = (0,)) -> List[Dict[str, int]]:
    return [{"full_block_cap": int(f), "subset_block_cap": int(s), "pass_form": int(p),
             "chain_passes": int(q)}
            for q in launches for p in forms for f in full_caps for s in subset_caps]


def _best(sweep: Dict[str, float], cands: List[Dict[str, int]]) -> dict:
    key = min(sweep, key=sweep.get)
    best = dict(cands[[_label(c) for c in cands].index(key)])
    best["ms"] = sweep[key]
    best["sweep_ms"] = sweep
    return best


def _label(c: Dict[str, int]) -> str:
    return (f"full={c['full_block_cap']},subset={c['subset_block_cap']},form={c['pass_form']},"
            f"chain={c.get('chain_passes', 0)}")


def tune_single(grid, optics, spots, iterations: int, compression: float, seed: int = 0,
                precision: str = "fp32", reps: int = 5, subset_caps=SUBSET_CAPS,
                full_caps=(0,), forms=PASS_FORMS, launches=LAUNCHES, stream=None) -> dict:
    """Fastest geometry for one hologram at a time of this shape."""
    import numpy as np
    import torch
    hg = _hg()
    stream = stream or torch.cuda.current_stream()
    dev = torch.tensor(np.stack([np.asarray(spots.x_mm), np.asarray(spots.y_mm),
                                 np.asarray(spots.z_mm), np.asarray(spots.amp)]),
                       dtype=torch.float64, device="cuda")
    phi = torch.empty(grid.W * grid.H, dtype=torch.float32, device="cuda")
    cands = _candidates(subset_caps, full_caps, forms, launches)
    sweep = {}
    for c in cands:
        sweep[_label(c)] = _time(lambda: hg.cswgs_device(
            grid, optics, dev, iterations, compression, seed, phi=phi, stream=stream,
            precision=precision, tune=c), reps, stream)
    return _best(sweep, cands)


def tune_batch(jobs, reps: int = 3, subset_caps=SUBSET_CAPS, full_caps=(0,), forms=PASS_FORMS,
               stream=None, use_graph: bool = True) -> dict:
    """Fastest geometry for a batch of DeviceJob run together."""
    import torch
    hg = _hg()
    stream = stream or torch.cuda.current_stream()
    cands = _candidates(subset_caps, full_caps, forms)
    sweep = {}
    for c in cands:
        batch = hg.Batch(jobs, tune=c, use_graph=use_graph)
        try:
            sweep[_label(c)] = _time(lambda: batch.run(stream), reps, stream)
        finally:
            batch.close()
    return _best(sweep, cands)


class Table:
    """JSON cache of tuned geometries keyed by workload shape."""

    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.entries: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def save(self) -> None:
        if not self.path:
            return
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    @staticmethod
    def as_tune(entry: dict) -> Dict[str, int]:
        return {"full_block_cap": int(entry["full_block_cap"]),
                "subset_block_cap": int(entry["subset_block_cap"]),
                "pass_form": int(entry.get("pass_form", 0)),
                "chain_passes": int(entry.get("chain_passes", 0))}

    def single(self, grid, optics, spots, iterations: int, compression: float,
               precision: str = "fp32", **kw) -> Dict[str, int]:
        key = single_key(grid, spots.n, iterations, compression, precision)
        if key not in self.entries:
            self.entries[key] = tune_single(grid, optics, spots, iterations, compression,
                                            precision=precision, **kw)
            self.save()
        return self.as_tune(self.entries[key])

    def batch(self, jobs, **kw) -> Dict[str, int]:
        key = batch_key(jobs)
        if key not in self.entries:
            self.entries[key] = tune_batch(jobs, **kw)
            self.save()
        return self.as_tune(self.entries[key])
