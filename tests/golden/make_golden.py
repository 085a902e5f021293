"""Writes the stored oracle results used by the full-size GPU parity tests.

Runs only the FP64 oracle (oracle/) on seeded synthetic inputs from
workload/; nothing here touches the GPU library.

    python tests/golden/make_golden.py [name ...]

Each case writes tests/golden/<name>.json holding e, u, the spot
intensities of the final hologram, the trajectory of the iterations (the
spot field V^j of every iteration j, and the weights w^j and phases theta^j
its update produces; V1 repeats V^1), and the final hologram Phi^I at a
fixed sample of pixels.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workload import Grid, OPTICS, PUPIL_OPTICS, spot_cloud  # noqa: E402

CASES = {
    # 1152 x 1152, N = 100, I = 30, CS-WGS with c = 1/16 and plain WGS.
    "cswgs_1152x1152_n100_i30_c16_seed0": dict(W=1152, H=1152, n=100, I=30, c=1 / 16, seed=0),
    "wgs_1152x1152_n100_i30_seed0": dict(W=1152, H=1152, n=100, I=30, c=None, seed=0),
    # 1920 x 1152 panel, 150 spots, deeper z range, CS-WGS with 20 iterations
    "cswgs_1920x1152_n150_i20_c16_seed3": dict(W=1920, H=1152, n=150, I=20, c=1 / 16, seed=3,
                                               z_half_mm=0.1),
    # the headline case under the paper's pupil: Gaussian illumination of
    # waist radius 6 mm on the round aperture 1152 pixels across
    "cswgs_1152x1152_n100_i30_c16_pupil_seed0": dict(W=1152, H=1152, n=100, I=30, c=1 / 16,
                                                     seed=0, pupil=True),
}

SAMPLE = 4096


def run(name: str, W, H, n, I, c, seed, z_half_mm=0.05, pupil=False):
    g = Grid(W, H)
    optics = PUPIL_OPTICS if pupil else OPTICS
    s = spot_cloud(seed, n, g, z_half_mm=z_half_mm)
    tr = oracle.Trace()
    t0 = time.time()
    if c is None:
        Phi = oracle.wgs(g, optics, s, I, seed, tr)
    else:
        Phi = oracle.cswgs(g, optics, s, I, c, seed, tr)
    e, u, inten = oracle.metrics(g, optics, s, Phi)
    rng = np.random.Generator(np.random.PCG64(12345))
    pix = np.sort(rng.choice(g.M, SAMPLE, replace=False))
    out = dict(
        W=W, H=H, n=n, iterations=I, compression=c, seed=seed, z_half_mm=z_half_mm,
        waist_mm=optics.waist_mm, aperture_px=optics.aperture_px,
        cloud="workload.spot_cloud(seed, n, Grid(W, H), z_half_mm=z_half_mm)",
        e=e, u=u, intensities=inten.tolist(),
        V1=[[float(v.real), float(v.imag)] for v in tr.V[0]],
        V=[[[float(v.real), float(v.imag)] for v in Vj] for Vj in tr.V],
        w=[[float(x) for x in wj] for wj in tr.w],
        theta=[[float(x) for x in tj] for tj in tr.theta],
        sample_pixels=pix.tolist(), sample_phi=Phi[pix].tolist(),
        oracle_seconds=time.time() - t0,
    )
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)
    print(name, "e", e, "u", u, "seconds", round(out["oracle_seconds"], 1), flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        run(nm, **CASES[nm])
