#!/usr/bin/env python3
"""Benchmark of the CS-WGS hologram hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--form fp32] [--no-cpu-baseline]

One step is one complete hologram: RS start, 30 CS-WGS iterations (forward
projection on a 1/16 random pixel subset for iterations 1..29, on all pixels
for iteration 30, weight update, back-propagation) and the final full-grid
phase, for a 1152 x 1152 SLM and 100 spots.  Spot clouds are synthetic
(seeded uniform clouds, workload/spots.py) and already resident in HBM when
the timed region starts; each step uses a different cloud and seed.

Printed: one JSON line with holograms/s, the roofline of the dominant kernel
measured live with HIP events on its stream, the accuracy of the seed-0
hologram against the stored FP64 oracle result, and the FP64 oracle timed
on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "holograms/s at M=1152^2,N=100 CS-WGS (e,u vs FP64 oracle); % FP32 roofline"
WORKLOAD = "cswgs_1152x1152_n100_i30_c16"
W = H = 1152
N = 100
ITER = 30
COMP = 1.0 / 16
CLOUDS = 10

# Algorithmic work of one (pixel, spot) term, FP32 flops (sincos counted
# separately): back-propagation 3 FMA for the phase + 2 FMA for the
# amplitude-weighted sum = 10; forward 3 FMA-equivalents for the phase +
# 4 FMA for the complex accumulate = 14.  The fused kernel does one of each
# per (pixel, spot) pair.
FLOPS_BACK = 10
FLOPS_FWD = 14
# Roofline of the per-pixel passes: plain FP32 vector ALU work (phases,
# v_fract_f32, v_sin_f32 / v_cos_f32, FMAs), reported against MI355X's
# published FP32 vector peak, 157.3 TFLOP/s = 256 CU x 2.4 GHz x 128 FMA
# lanes per clock per CU = 78.65 T FMA/s.  The microbenchmark
# paper_2003_05293_amd/bench_alu (built without packed FP32 instructions)
# measures non-packed FP32 operations at up to 0.89 of that issue rate
# (v_fract_f32 + v_add_f32: 70.3 T/s; v_fmamk_f32 chains: 55.3 T/s), so the
# published rate is the ceiling of this code as it is, and the transcendentals
# at a quarter of it (19.0 and 19.4 T/s).
PEAK_FP32_TFLOPS = 157.3
ISSUE_T_PER_S = 256 * 2.4e9 * 128 / 1e12
# Side figure: the issue-limited peak of the algorithm's own instruction mix.
# A (pixel, spot) pair of the two-sincos pass issues 3 FMA + fract + sin +
# cos + 2 FMA (back-propagation) and 3 FMA + fract + sin + cos + 4 FMA
# (forward): 12 FMA + 2 fract + 4 transcendentals at four slots each = 30
# full-rate slots, so at most 78.65 / 30 = 2.62 T pairs/s, i.e. 62.9 TFLOP/s
# at 24 algorithmic flops per pair.
SLOTS_PER_PAIR = 12 + 2 + 4 * 4
PEAK_ISSUE_TFLOPS = round(ISSUE_T_PER_S / SLOTS_PER_PAIR * (FLOPS_BACK + FLOPS_FWD), 1)
# Launch tags of the library's kernel timing (hg_timing_read).
KERNELS = ("k_prologue", "k_perm", "k_sep_pass", "k_sep_final", "k_pass_subset",
           "k_pass_full", "k_pass_mixed", "k_backprop_phi", "k_mxp_subset",
           "k_mx_full", "k_mx_final")


# HBM traffic of the dominant kernel per launch, from the rocprofv3 PMC
# summary committed under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled
# by what the same counter reads for a copy of known size).  It holds only
# while the kernel's sources are those the counters were taken on.
TRAFFIC_SOURCES = ("kernels.hip", "kernels.hpp", "pass_tail.hpp", "device_common.hpp",
                   "device_math.hpp")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2003_05293_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(kernel: str):
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{WORKLOAD}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-json:"):
                t = json.loads(line[len("traffic-json:"):])
                if t.get("sources_sha256") != kernel_sources_sha256():
                    return None
                return round(1024.0 * (t["fetch_kib"] * t["fetch_scale"]
                                       + t["write_kib"] * t["write_scale"]))
    return None


# ------------------------------------------------- CPU baseline (oracle) ---
# The FP64 oracle on the host cores, as it stands: one process, and a pool of
# worker processes over a fixed partition of the pixel set into blocks of
# CPU_BLOCK consecutive entries, whose results are combined in block order
# (the same numbers whatever the number of workers).  Workers are forked
# before the GPU is touched and use one BLAS thread each.
CPU_BLOCK = 4096
CPU_MAX_WORKERS = 16  # the host share of one GPU
_CPU_CTX = None  # (grid, optics, spots) of the current job, inherited by the workers


def _one_thread():
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except Exception:  # pragma: no cover
        return None


def _cpu_back_block(args):
    import oracle
    w, th, p = args
    g, o, s = _CPU_CTX
    return oracle.backward(g, o, s, w, th, p)


def _cpu_fwd_block(args):
    import oracle
    phi, p = args
    g, o, s = _CPU_CTX
    return oracle.forward(g, o, s, phi, p) * p.shape[0]  # the block's sum


class _OracleRunner:
    """eq. (1) and eq. (3) of the oracle on a pixel set, in one process
    (pool None) or over the fixed blocks of a pool."""

    def __init__(self, pool):
        self.pool = pool

    def backward(self, w, th, p):
        import oracle
        g, o, s = _CPU_CTX
        if self.pool is None:
            return oracle.backward(g, o, s, w, th, p)
        parts = self.pool.map(_cpu_back_block, [(w, th, p[k:k + CPU_BLOCK])
                                                for k in range(0, p.shape[0], CPU_BLOCK)])
        return np.concatenate(parts)

    def forward(self, phi, p):
        import oracle
        g, o, s = _CPU_CTX
        if self.pool is None:
            return oracle.forward(g, o, s, phi, p)
        parts = self.pool.map(_cpu_fwd_block, [(phi[k:k + CPU_BLOCK], p[k:k + CPU_BLOCK])
                                               for k in range(0, p.shape[0], CPU_BLOCK)])
        V = parts[0].copy()
        for v in parts[1:]:
            V += v
        return V / p.shape[0]

    def wgs(self, grid, spots, iterations, seed):
        """RS, then `iterations` full iterations: the oracle's WGS steps."""
        import oracle
        allp = np.arange(grid.M, dtype=np.int64)
        w, th = np.ones(spots.n), oracle.theta0(seed, spots.n)
        Phi = self.backward(w, th, allp)
        for _ in range(iterations):
            w, th = oracle.update(w, self.forward(Phi, allp))
            Phi = self.backward(w, th, allp)
        return Phi

    def cswgs_sample(self, grid, spots, seed):
        """The bounded sample of one headline hologram: one full-grid
        back-propagation, one full-grid forward projection and two compressed
        iterations; returns the seconds of each part."""
        import oracle
        allp = np.arange(grid.M, dtype=np.int64)
        w, th = np.ones(spots.n), oracle.theta0(seed, spots.n)
        t0 = time.perf_counter()
        Phi = self.backward(w, th, allp)
        t_fb = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.forward(Phi, allp)
        t_ff = time.perf_counter() - t0
        t0 = time.perf_counter()
        for j in (1, 2):
            p = oracle.sampler.subset(grid.M, oracle.sampler.ORDER_KEY, j, COMP)
            V = self.forward(self.backward(w, th, p), p)
            w, th = oracle.update(w, V)
        t_sub = (time.perf_counter() - t0) / 2
        return t_fb, t_ff, t_sub


def cpu_baseline(grid, optics, spots, seed):
    """Times the FP64 oracle on the host cores, single-process and across a
    pool of workers: on a bounded sample of one headline hologram (scaled to
    the whole hologram: the oracle computes the phase on all pixels for the
    last two iterations and on the next window otherwise, so a hologram is
    2 full back-propagations + 1 full forward projection + 29 compressed
    iterations), and on the small WGS workload (256^2, N = 16, 20 iterations)
    in full.  Runs before the GPU is touched (the workers are forked)."""
    global _CPU_CTX
    import multiprocessing as mp
    from workload import Grid, spot_cloud
    affinity = len(os.sched_getaffinity(0))
    workers = max(1, min(affinity, CPU_MAX_WORKERS))
    small = Grid(256, 256)
    small_spots = spot_cloud(0, 16, small)
    legs = {}
    limiter = _one_thread()
    ctx = mp.get_context("fork")

    def timed(job, nproc, fn):
        # the workers are forked after the job's context is set
        global _CPU_CTX
        _CPU_CTX = job
        pool = None if nproc == 1 else ctx.Pool(nproc, initializer=_one_thread)
        try:
            return fn(_OracleRunner(pool))
        finally:
            if pool is not None:
                pool.close()
                pool.join()

    def run_small(run):
        t0 = time.perf_counter()
        run.wgs(small, small_spots, 20, 0)
        return time.perf_counter() - t0

    for name, nproc in (("one_core", 1), ("all_cores", workers)):
        t_fb, t_ff, t_sub = timed((grid, optics, spots), nproc,
                                  lambda run: run.cswgs_sample(grid, spots, seed))
        per_holo = 2 * t_fb + t_ff + (ITER - 1) * t_sub
        t_small = timed((small, optics, small_spots), nproc, run_small)
        legs[name] = {"holograms_per_s": 1.0 / per_holo, "s_per_hologram": round(per_holo, 3),
                      "processes": nproc, "full_back_s": round(t_fb, 3),
                      "full_forward_s": round(t_ff, 3), "compressed_iteration_s": round(t_sub, 4),
                      "wgs_256x256_n16_i20_s": round(t_small, 3)}
        print(f"[bench] oracle {name} ({nproc} processes): {per_holo:.2f} s per headline "
              f"hologram, 256^2 WGS in {t_small:.2f} s", file=sys.stderr, flush=True)
    _CPU_CTX = None
    if limiter is not None:
        limiter.unregister()
    best = legs["all_cores"]
    return {
        "value": best["holograms_per_s"], "unit": "holograms/s", "cores": workers,
        "affinity_cores": affinity, "kind": "oracle",
        "sample": (f"seed-{seed} headline hologram: 1 full back-propagation, 1 full forward and "
                   f"2 compressed iterations, scaled to 2 full back + 1 full forward + "
                   f"{ITER - 1} compressed iterations; {workers} worker processes over fixed "
                   f"blocks of {CPU_BLOCK} pixels; plus WGS on 256^2, N=16, 20 iterations in full"),
        "legs": legs,
    }


def kernel_times(hg, run, count):
    """Per-family kernel durations (HIP events on the launch stream) over
    `count` calls of run(k)."""
    import torch
    hg.timing_reset()
    hg.timing_enable(True)
    for k in range(count):
        run(k)
    torch.cuda.synchronize()
    hg.timing_enable(False)
    kern = {}
    for name in KERNELS:
        ms, cnt = hg.timing_read(name)
        if cnt:
            kern[name] = {"total_ms": ms, "launches": cnt, "avg_us": 1000.0 * ms / cnt}
    return kern


def single_form(hg, grid, clouds, spots_dev, phis, stream, form, steps, warmup, gold, tune,
                optics=None, label=None):
    """One hologram per call on one stream in the given precision (and
    optics: the uniform full grid by default), with its e, u error against
    the stored FP64 oracle result of the seed-0 cloud."""
    import torch
    from workload import OPTICS
    if optics is None:
        optics = OPTICS
    for k in range(warmup):
        hg.cswgs_device(grid, optics, spots_dev[k % CLOUDS], ITER, COMP, k % CLOUDS,
                        phi=phis[k % CLOUDS], stream=stream, precision=form, tune=tune)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for k in range(steps):
        hg.cswgs_device(grid, optics, spots_dev[k % CLOUDS], ITER, COMP, k % CLOUDS,
                        phi=phis[k % CLOUDS], stream=stream, precision=form, tune=tune)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    kern = kernel_times(hg, lambda k: hg.cswgs_device(
        grid, optics, spots_dev[k % CLOUDS], ITER, COMP, k % CLOUDS, phi=phis[k % CLOUDS],
        stream=stream, precision=form, tune=tune), min(steps, 10))
    hg.cswgs_device(grid, optics, spots_dev[0], ITER, COMP, 0, phi=phis[0], stream=stream,
                    precision=form, tune=tune)
    e, u, _ = hg.metrics(grid, optics, clouds[0], phis[0])
    out = {"holograms_per_s": round(1000.0 / ms, 3), "ms_per_hologram": round(ms, 5),
           "how": "one hologram per call, back to back on one stream", "e": e, "u": u,
           "kernels": {k: {"avg_us": round(v["avg_us"], 3), "launches_per_hologram":
                           v["launches"] / min(steps, 10)} for k, v in kern.items()}}
    if gold is not None:
        out.update({"e_abs_err": abs(e - gold["e"]), "u_abs_err": abs(u - gold["u"])})
    print(f"[bench] {label or form}: {ms:.4f} ms per hologram, e {e:.6f} u {u:.6f}",
          file=sys.stderr, flush=True)
    return out


def _time_batch(torch, batch, stream, runs):
    batch.run(stream)
    stream.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(runs):
        batch.run(stream)
    b.record(stream)
    stream.synchronize()
    return a.elapsed_time(b) / runs


def batched_forms(hg, grid, optics, steps, bsize):
    """Batched forms: `bsize` holograms of the headline size (distinct
    clouds and seeds) in one graph-captured batch, and the 64-hologram mixed
    batch (sizes 512^2 .. 1920x1152, N in [8, 200], z within +-0.1 mm)."""
    import numpy as np
    import torch
    from workload import spot_cloud, mixed_batch
    stream = torch.cuda.Stream()
    out = {}
    jobs = [hg.DeviceJob.from_spots(grid, optics, spot_cloud(100 + k, N, grid), ITER, COMP,
                                    100 + k) for k in range(bsize)]
    from paper_2003_05293_amd import autotune
    tuned = autotune.tune_batch(jobs, reps=2, stream=stream)
    batch = hg.Batch(jobs, tune=autotune.Table.as_tune(tuned), use_graph=True)
    runs = max(1, steps // bsize + 1)
    ms = _time_batch(torch, batch, stream, runs)
    out["fp32_batched"] = {"holograms_per_s": round(1000.0 * bsize / ms, 3),
                           "ms_per_batch": round(ms, 4), "batch": bsize, "runs": runs,
                           "tune": autotune.Table.as_tune(tuned),
                           "how": f"{bsize} holograms of this workload per graph-captured batch"}
    print(f"[bench] batched x{bsize}: {ms:.3f} ms per batch", file=sys.stderr, flush=True)
    batch.close()
    del jobs
    mixed = mixed_batch(0, count=64)
    mjobs = [hg.DeviceJob.from_spots(j.grid, optics, j.spots, j.iterations, j.compression, j.seed)
             for j in mixed]
    terms = sum((j.grid.M * 3 + 2 * (j.iterations - 1) * math.ceil(j.compression * j.grid.M))
                * j.spots.n for j in mixed)
    tuned = autotune.tune_batch(mjobs, reps=2, stream=stream)
    batch = hg.Batch(mjobs, tune=autotune.Table.as_tune(tuned), use_graph=True)
    ms = _time_batch(torch, batch, stream, 3)
    out["fp32_mixed64"] = {"holograms_per_s": round(64000.0 / ms, 3), "ms_per_batch": round(ms, 4),
                           "terms_per_s": round(terms / (ms * 1e-3), 1),
                           "tune": autotune.Table.as_tune(tuned),
                           "how": "64 mixed holograms (sizes 512^2..1920x1152, N 8..200, I 30, "
                                  "c 1/16) per graph-captured batch"}
    print(f"[bench] mixed64: {ms:.3f} ms per batch", file=sys.stderr, flush=True)
    batch.close()
    return out


SWEEP_RATES = (60, 250, 500, 1000, 1500, 2000, 3000, 4000)
SWEEP_S = 3.0
SWEEP_P99_MS = 50.0


def served_form(hg, optics, seconds):
    """Served form: Poisson arrivals at 60 requests/s (N uniform in [10, 150],
    1152^2 or 1920x1152, CS-WGS 20 iterations, c = 1/16) replayed in real time
    through the continuous-batching engine."""
    import torch
    from paper_2003_05293_amd import serve
    from workload import poisson_stream
    reqs = poisson_stream(0, rate_hz=60.0, duration_s=seconds, iterations=20)
    stream = torch.cuda.Stream()
    eng = hg.Engine(16 << 30, max_slots=64)
    warm = poisson_stream(1, rate_hz=60.0, duration_s=0.5, iterations=20)
    serve.replay(warm, optics, eng, stream)
    res = serve.replay(reqs, optics, eng, stream)
    eng.close()
    print(f"[bench] served {res.completed} requests in {res.wall_s:.2f} s, p50 "
          f"{1e3 * res.percentile(50):.3f} ms, p99 {1e3 * res.percentile(99):.3f} ms",
          file=sys.stderr, flush=True)
    # offered-load sweep: the same request mix at rising Poisson rates, each
    # for SWEEP_S seconds, until p99 breaks SWEEP_P99_MS (or the completion
    # rate falls below 90 % of the offered rate)
    sweep = []
    for k, rate in enumerate(SWEEP_RATES):
        rq = poisson_stream(10 + k, rate_hz=rate, duration_s=SWEEP_S, iterations=20)
        eng = hg.Engine(16 << 30, max_slots=64)
        r = serve.replay(rq, optics, eng, stream)
        eng.close()
        row = {"offered_per_s": rate, "requests": len(rq),
               "completed_per_s": round(r.completed / r.wall_s, 1),
               "p50_ms": round(1e3 * r.percentile(50), 3), "p99_ms": round(1e3 * r.percentile(99), 3),
               "engine_steps": r.steps}
        sweep.append(row)
        print(f"[bench] served at {rate}/s: {row['completed_per_s']}/s, p50 {row['p50_ms']} ms, "
              f"p99 {row['p99_ms']} ms", file=sys.stderr, flush=True)
        if row["p99_ms"] > SWEEP_P99_MS or row["completed_per_s"] < 0.9 * rate:
            break
    within = [x for x in sweep if x["p99_ms"] <= SWEEP_P99_MS and x["completed_per_s"] >= 0.9 * x["offered_per_s"]]
    return {"holograms_per_s": round(res.completed / res.wall_s, 3),
            "offered_per_s": 60.0, "requests": len(reqs), "completed": res.completed,
            "p50_ms": round(1e3 * res.percentile(50), 4), "p99_ms": round(1e3 * res.percentile(99), 4),
            "engine_steps": res.steps, "seconds": seconds,
            "how": "Poisson 60/s, N in [10,150], 1152^2 or 1920x1152, I 20, c 1/16, "
                   "continuous batching, latency arrival -> observed completion",
            "load_sweep": sweep,
            "saturation": {"p99_bound_ms": SWEEP_P99_MS,
                           "highest_rate_within_bound": within[-1]["offered_per_s"] if within else None,
                           "completed_per_s_there": within[-1]["completed_per_s"] if within else None},
            "load_sweep_how": f"same request mix, {SWEEP_S} s per rate, rates rising until p99 > "
                              f"{SWEEP_P99_MS} ms or completions < 90 % of the offered rate"}


def slm_output(hg, grid, spots_dev, phis, stream, tune, steps):
    """The SLM's gray image: the headline hologram with the lookup fused into
    its final pass, and the standalone conversion of a hologram (HBM-bound:
    4 bytes read and 1 written per pixel), timed with HIP events."""
    import numpy as np
    import torch
    from workload import OPTICS
    table = np.rint(255 * (np.arange(256) / 255.0) ** 0.8).astype(np.uint16)
    lut = hg.Lut(table, bits=8)
    gray = lut.new_image(grid)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    params = dict(phi=phis[0], stream=stream, tune=tune)
    for k in range(3):
        hg.cswgs_device(grid, OPTICS, spots_dev[k % CLOUDS], ITER, COMP, k % CLOUDS, **params)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        hg.cswgs_device(grid, OPTICS, spots_dev[k % CLOUDS], ITER, COMP, k % CLOUDS,
                        lut=lut, gray=gray, **params)
    ev[1].record(stream)
    reps = 200
    for _ in range(5):
        hg.phase_to_gray(lut, phis[0], gray=gray, stream=stream)
    ev[2].record(stream)
    for _ in range(reps):
        hg.phase_to_gray(lut, phis[0], gray=gray, stream=stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    fused_ms = ev[0].elapsed_time(ev[1]) / steps
    conv_us = 1000.0 * ev[2].elapsed_time(ev[3]) / reps
    bytes_ = 5 * grid.W * grid.H
    lut.close()
    print(f"[bench] SLM gray: fused {fused_ms:.4f} ms per hologram, "
          f"standalone {conv_us:.2f} us", file=sys.stderr, flush=True)
    return {"fused_ms_per_hologram": round(fused_ms, 5),
            "phase_to_gray_us": round(conv_us, 3),
            "phase_to_gray_GBps": round(bytes_ / (conv_us * 1e-6) / 1e9, 1),
            "how": "8-bit table of 256 levels; fused: the headline hologram with the gray "
                   "image written by its final pass; standalone: "
                   "hg_phase_to_gray of one 1152^2 hologram, back to back, 5 bytes per pixel"}



def budget_sweep(hg):
    """The paper's algorithm comparison at a fixed amount of work, on the
    scenario stand-ins at 1152^2 under the paper's pupil (10 orientations and
    theta^0 each); e and u as mean +- std, and the GPU time per hologram."""
    from paper_2003_05293_amd import budget
    from workload import Grid, PUPIL_OPTICS
    t0 = time.perf_counter()
    res = budget.sweep(Grid(W, H), PUPIL_OPTICS, ("grid100", "grid36", "cubes"), repeats=10)
    out = {}
    for name, rows in res.items():
        out[name] = [{"algorithm": r["algorithm"], "c": r["compression"], "I": r["iterations"],
                      "e": [round(r["e"]["mean"], 5), round(r["e"]["std"], 5)],
                      "u": [round(r["u"]["mean"], 5), round(r["u"]["std"], 5)],
                      "ms_per_hologram": round(r["ms_per_hologram"], 4)} for r in rows]
    print(f"[bench] budget sweep: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return {"budget_terms_per_pixel": budget.BUDGET_TERMS_PER_PIXEL, "repeats": 10,
            "grid": [W, H], "optics": "pupil: waist 6 mm, aperture 1152 px",
            "how": "every algorithm at the largest iteration count within the budget of "
                   "(pixel, spot) terms; e, u mean and std over 10 orientations and theta^0",
            "results": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--form", default="fp32", choices=["fp32", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch", type=int, default=32, help="holograms per batched launch")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the served Poisson stream (0: skip)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline workload only (no other forms, sweep or CPU leg); "
                         "for profiling runs")
    ap.add_argument("--no-budget-sweep", action="store_true",
                    help="skip the fixed-work comparison of RS, WGS and CS-WGS on the scenarios")
    ap.add_argument("--no-autotune", action="store_true",
                    help="default launch parameters instead of the autotuned ones")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device three times (counter calibration) "
                         "and exit")
    args = ap.parse_args()
    if args.headline_only:
        args.no_batched = args.no_budget_sweep = args.no_cpu_baseline = True
        args.serve_seconds = 0.0
    if args.calibrate_copy > 0:
        import torch
        n = args.calibrate_copy << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read_per_copy": 4 * n,
                          "calibrate_copy_bytes_written_per_copy": 4 * n, "copies": 3}))
        return
    # Python's cyclic garbage collector is off for the whole run: its full
    # collections (one every ~200 hologram calls here, from the binding's
    # per-call ctypes objects) stall the host for 45-60 ms, long enough to
    # starve the GPU; the objects are freed by reference counting anyway.
    gc.collect()
    gc.freeze()
    gc.disable()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the hologram "
              "path has no multi-GPU form in this build", file=sys.stderr)
        sys.exit(2)

    from workload import Grid, OPTICS, spot_cloud
    grid = Grid(W, H)
    clouds = [spot_cloud(s, N, grid) for s in range(CLOUDS)]
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host cores", file=sys.stderr, flush=True)
        cpu = cpu_baseline(grid, OPTICS, clouds[0], 0)

    import torch
    import paper_2003_05293_amd as hg
    spots_dev = [torch.tensor(np.stack([c.x_mm, c.y_mm, c.z_mm, c.amp]), dtype=torch.float64,
                              device="cuda") for c in clouds]
    phis = [torch.empty(W * H, dtype=torch.float32, device="cuda") for _ in range(CLOUDS)]
    stream = torch.cuda.current_stream()

    # launch geometry of the compressed passes, chosen by the autotuner
    from paper_2003_05293_amd import autotune
    if args.no_autotune:
        tuned = {"full_block_cap": 0, "subset_block_cap": 0, "pass_form": 0, "ms": None,
                 "sweep_ms": {}}
    else:
        tuned = autotune.tune_single(grid, OPTICS, clouds[0], ITER, COMP, precision="fp32", reps=5)
    tune = autotune.Table.as_tune(tuned)
    print(f"[bench] launch parameters {tune} ({tuned['ms']} ms)", file=sys.stderr, flush=True)

    def step(k):
        s = k % CLOUDS
        hg.cswgs_device(grid, OPTICS, spots_dev[s], ITER, COMP, s, phi=phis[s], stream=stream,
                        precision=args.form, tune=tune)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} holograms)", file=sys.stderr, flush=True)

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(k)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = start.elapsed_time(stop) / args.steps
    value = 1000.0 / ms_per_step
    print(f"[bench] timed {args.steps} holograms: {ms_per_step:.4f} ms each", file=sys.stderr,
          flush=True)

    # Dominant kernel, timed live with HIP events on the stream it runs on.
    hg.timing_reset()
    hg.timing_enable(True)
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    hg.timing_enable(False)
    kern = {}
    for name in KERNELS:
        ms, cnt = hg.timing_read(name)
        if cnt:
            kern[name] = {"total_ms": ms, "launches": cnt, "avg_us": 1000.0 * ms / cnt}
    dominant = max(kern, key=lambda k: kern[k]["total_ms"])
    m = math.ceil(COMP * W * H)
    # (pixel, spot) pairs per launch and the steps each launch performs
    pairs = {"k_pass_subset": (m, FLOPS_BACK + FLOPS_FWD),
             "k_pass_chain": (m * (ITER - 1), FLOPS_BACK + FLOPS_FWD),
             "k_pass_full": (W * H, FLOPS_BACK + FLOPS_FWD),
             "k_sep_pass": (W * H, FLOPS_BACK + FLOPS_FWD),
             "k_sep_final": (W * H, FLOPS_BACK),
             "k_backprop_phi": (W * H, FLOPS_BACK),
             "k_mxp_subset": (m, FLOPS_BACK + FLOPS_FWD),
             "k_mx_full": (W * H, FLOPS_BACK + FLOPS_FWD),
             "k_mx_final": (W * H, FLOPS_BACK)}
    if dominant not in pairs:
        raise RuntimeError(f"dominant kernel {dominant} has no algorithmic flop count")
    px, fl = pairs[dominant]
    flops = px * N * fl
    achieved = flops / (kern[dominant]["avg_us"] * 1e-6) / 1e12
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
        "traffic": profiled_traffic(dominant),
        "peak_basis": "MI355X published FP32 vector peak",
        "peak_issue_derived": PEAK_ISSUE_TFLOPS,
        "frac_of_issue_derived": round(achieved / PEAK_ISSUE_TFLOPS, 4),
        "issue_derived_basis": f"{SLOTS_PER_PAIR} full-rate issue slots per (pixel, spot) pair "
                               f"(12 FMA, 2 fract, 4 sin/cos at quarter rate) at "
                               f"{ISSUE_T_PER_S:.2f} T slots/s",
        "kernel": dominant, "avg_launch_us": round(kern[dominant]["avg_us"], 3),
        "flops_per_launch": flops,
        "kernels": {k: {"avg_us": round(v["avg_us"], 3),
                        "launches_per_hologram": v["launches"] / args.steps}
                    for k, v in kern.items()},
    }

    # Accuracy of the seed-0 hologram against the stored FP64 oracle run.
    accuracy = None
    gold = os.path.join(ROOT, "tests", "golden", "cswgs_1152x1152_n100_i30_c16_seed0.json")
    gd = None
    if os.path.exists(gold):
        with open(gold) as f:
            gd = json.load(f)
    step(0)
    e, u, _ = hg.metrics(grid, OPTICS, clouds[0], phis[0])
    accuracy = {"e": e, "u": u}
    if gd is not None:
        accuracy.update({"e_oracle": gd["e"], "u_oracle": gd["u"],
                         "e_abs_err": abs(e - gd["e"]), "u_abs_err": abs(u - gd["u"])})

    forms = {args.form: {"holograms_per_s": round(value, 3),
                         "ms_per_hologram": round(ms_per_step, 5),
                         "how": "one hologram per call, back to back on one stream"}}
    other = "mixed" if args.form == "fp32" else "fp32"
    if not args.headline_only:
        forms[other] = single_form(hg, grid, clouds, spots_dev, phis, stream, other, args.steps,
                                   args.warmup, gd, tune)
    # the same workload under the paper's pupil (Gaussian illumination of
    # 6 mm waist on the round 1152-pixel aperture)
    from workload import PUPIL_OPTICS
    pgold = os.path.join(ROOT, "tests", "golden", "cswgs_1152x1152_n100_i30_c16_pupil_seed0.json")
    pgd = None
    if os.path.exists(pgold):
        with open(pgold) as f:
            pgd = json.load(f)
    if not args.headline_only:
        forms["fp32_pupil"] = single_form(hg, grid, clouds, spots_dev, phis, stream, "fp32",
                                          args.steps, args.warmup, pgd, tune,
                                          optics=PUPIL_OPTICS, label="fp32 pupil")
        forms["fp32_pupil"]["optics"] = {"waist_mm": PUPIL_OPTICS.waist_mm,
                                         "aperture_px": PUPIL_OPTICS.aperture_px}
    if not args.no_batched:
        forms.update(batched_forms(hg, grid, OPTICS, args.steps, args.batch))
    if args.serve_seconds > 0:
        forms["fp32_served"] = served_form(hg, OPTICS, args.serve_seconds)

    slm = None if args.headline_only else slm_output(hg, grid, spots_dev, phis, stream, tune,
                                                      args.steps)

    sweep = None
    if not args.no_budget_sweep:
        sweep = budget_sweep(hg)

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "holograms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "wall_s": round(wall, 4),
        "config": {"workload": WORKLOAD, "W": W, "H": H, "N": N, "iterations": ITER,
                   "compression": COMP, "form": args.form, "clouds": CLOUDS,
                   "spots": "resident in HBM", "tune": tune,
                   "tune_sweep_ms": {k: round(v, 4) for k, v in tuned["sweep_ms"].items()}},
        "roofline": roofline, "accuracy": accuracy, "forms": forms, "cpu_baseline": cpu,
        "slm_output": slm, "budget_sweep": sweep,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
