"""Fixed-budget comparison of RS, WGS and CS-WGS (paper, results section).

The paper compares the algorithms at a fixed frame time: within 64 ms on
its GPU, WGS fits a single iteration for the 100-spot grid and five for the
36-spot grid, while CS-WGS at compression c fits many more.  On a machine
whose cost is proportional to the number of (pixel, spot) terms evaluated,
a fixed time is a fixed number of terms, so the comparison is reproduced on
any hardware by fixing the work instead of the time:

    RS           M N
    WGS, I       (2 I + 1) M N
    CS-WGS, I    2 (I - 1) m N + 3 M N,   m = ceil(c M)   (I >= 2)

(CS-WGS: Phi^0 and Phi^1..Phi^{I-2} on the next window, the forward sums of
iterations 1..I-1 on their windows, then Phi^{I-1}, the last forward sum and
Phi^I on all M pupil pixels.  The paper's own linear estimate,
2 M N + c M N (I - 2), counts the same schedule with one term per pixel and
spot per iteration.)  A budget of B = 432 M terms gives WGS one iteration
at N = 100 (300 <= 432 < 500) and five at N = 36 (396 <= 432 < 468), the
paper's two anchors; every algorithm then runs the largest iteration count
that fits.

``sweep`` runs every scenario, algorithm and repeat through the library
(the seed of repeat k sets the scenario's orientation and theta^0), scores
each hologram with the FP64 metrics and times it with HIP events.  The
measured times show what the same work costs on this GPU.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

BUDGET_TERMS_PER_PIXEL = 432
COMPRESSIONS = tuple(2.0 ** -k for k in range(1, 9))
CONVERGED_ITERATIONS = 100


def terms(algorithm: str, M: int, N: int, iterations: int = 0,
          compression: Optional[float] = None) -> int:
    """(pixel, spot) terms of one hologram: algorithm 'rs', 'wgs' or 'cswgs'
    over M pupil pixels."""
    if algorithm == "rs":
        return M * N
    if algorithm == "wgs":
        return (2 * iterations + 1) * M * N
    if algorithm == "cswgs":
        if iterations < 2:
            return (2 * iterations + 1) * M * N
        m = math.ceil(compression * M)
        return 2 * (iterations - 1) * m * N + 3 * M * N
    raise ValueError(f"unknown algorithm {algorithm!r}")


def iterations_for_budget(algorithm: str, M: int, N: int, compression: Optional[float] = None,
                          budget_per_pixel: int = BUDGET_TERMS_PER_PIXEL) -> int:
    """Largest iteration count whose terms fit budget_per_pixel * M (0 when
    not even one iteration fits)."""
    budget = budget_per_pixel * M
    if algorithm == "wgs":
        return max(0, (budget // (M * N) - 1) // 2)
    if algorithm == "cswgs":
        if terms("wgs", M, N, 1) > budget:
            return 0
        m = math.ceil(compression * M)
        return 1 + (budget - 3 * M * N) // (2 * m * N)
    raise ValueError(f"unknown algorithm {algorithm!r}")


def _stats(vals: Sequence[float]) -> Dict[str, float]:
    n = len(vals)
    mean = sum(vals) / n
    var = sum((v - mean) ** 2 for v in vals) / (n - 1) if n > 1 else 0.0
    return {"mean": mean, "std": math.sqrt(var)}


def sweep(grid, optics, scenarios: Sequence[str], repeats: int = 10,
          compressions: Sequence[float] = COMPRESSIONS,
          budget_per_pixel: int = BUDGET_TERMS_PER_PIXEL,
          converged_iterations: int = CONVERGED_ITERATIONS, stream=None) -> Dict[str, List[dict]]:
    """e and u (mean and standard deviation over `repeats` orientations and
    theta^0) and the GPU time per hologram of RS, WGS and CS-WGS at every
    compression, each at the iteration count of the budget, plus WGS run to
    `converged_iterations` as the reference without a budget."""
    import torch

    import paper_2003_05293_amd as hg
    from workload import scenario

    if stream is None:
        stream = torch.cuda.current_stream()
    # pupil size: the number of pixels the full passes sum over
    M = _pupil_size(hg, grid, optics)
    phis = [torch.empty(grid.W * grid.H, dtype=torch.float32, device="cuda")
            for _ in range(repeats)]
    out: Dict[str, List[dict]] = {}
    for name in scenarios:
        clouds = [scenario(name, k, grid, optics) for k in range(repeats)]
        N = clouds[0].n
        configs = [("rs", None, 0),
                   ("wgs", None, iterations_for_budget("wgs", M, N,
                                                       budget_per_pixel=budget_per_pixel))]
        configs += [("cswgs", c, iterations_for_budget("cswgs", M, N, c, budget_per_pixel))
                    for c in compressions]
        configs.append(("wgs_converged", None, converged_iterations))
        rows = []
        for alg, c, I in configs:
            def run(k):
                if alg == "rs":
                    hg.rs(grid, optics, clouds[k], k, phi=phis[k], stream=stream)
                elif alg == "cswgs":
                    hg.cswgs(grid, optics, clouds[k], I, c, k, phi=phis[k], stream=stream)
                else:
                    hg.wgs(grid, optics, clouds[k], I, k, phi=phis[k], stream=stream)
            run(0)  # warm-up (workspace sizing)
            # the repeats back to back on the stream: GPU time per hologram
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            for k in range(repeats):
                run(k)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / repeats
            es, us = [], []
            for k in range(repeats):
                e, u, _ = hg.metrics(grid, optics, clouds[k], phis[k], stream=stream)
                es.append(e)
                us.append(u)
            kind = "cswgs" if alg == "cswgs" else ("rs" if alg == "rs" else "wgs")
            rows.append({"algorithm": alg, "compression": c, "iterations": I, "N": N,
                         "terms_per_pixel": terms(kind, M, N, I, c) / M,
                         "e": _stats(es), "u": _stats(us), "ms_per_hologram": ms})
        out[name] = rows
    return out


def _pupil_size(hg, grid, optics) -> int:
    """|Omega| as the library counts it: the length of its random order at
    compression 1 (the one subset that holds every pupil pixel)."""
    return int(hg.subset(grid, 0, 1, 1.0, optics=optics).shape[0])
