"""D3Q15 (the paper's NSE lattice) against D3Q19 (the other one it names,
Sec. II B after Eq. 22): accuracy against throughput.

* Static droplets (periodic boxes, FP64): the Laplace pressure jump against
  2 sigma / R_eff, R_eff from the droplet volume, and the largest spurious
  velocity, after `steps` steps.
* A Rayleigh-Taylor box (FP32): spike and bubble positions of the two
  lattices at the same times.
* Throughput of the FP32 step on the 256 x 256 x 1024 Rayleigh-Taylor box.
* The two study switches of the D3Q15 model on the 48^3 droplet: D3Q7 finite
  differences, and the untruncated forcing of Eq. 28.

One JSON line per result:

    python -m paper_1507_07294_amd.lattice_study
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import mplb
from . import workloads as wl


def _with_q(w, q):
    w.nse_q = q
    return w


def laplace_run(q, n=48, R=12.0, steps=3000, sigma=0.01, D=4.0, stencil=0, forcing=0):
    w = _with_q(wl.static_droplet(n=n, R=R, D=D, sigma=sigma), q)
    w.params = w.params.replace(stencil=stencil, forcing=forcing)
    lt = mplb.from_workload(w, "f64")
    lt.step(steps)
    phi, p = lt.read("phi"), lt.read("p")
    u = np.sqrt(lt.read("ux") ** 2 + lt.read("uy") ** 2 + lt.read("uz") ** 2)
    lt.destroy()
    c = n / 2.0
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    R_eff = (3.0 * ((1.0 + phi) / 2.0).sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    dp = p[r < R_eff - D].mean() - p[r > R_eff + D].mean()
    ref = 2.0 * sigma / R_eff
    return {"case": "laplace", "q": q, "stencil": "D3Q7" if stencil else "D3Q15",
            "forcing": "Eq. 28" if forcing else "Eq. 32", "n": n, "R": R, "steps": steps, "R_eff": round(R_eff, 4),
            "dp": float(f"{dp:.6e}"), "two_sigma_over_R": float(f"{ref:.6e}"),
            "laplace_rel_err": float(f"{abs(dp - ref) / ref:.4e}"), "max_spurious_u": float(f"{u.max():.4e}")}


def front_run(W=64, Re=256.0, checkpoints=(800, 1600)):
    out = []
    lats = {q: mplb.from_workload(_with_q(wl.rayleigh_taylor(W=W, Re=Re), q), "f32") for q in (15, 19)}
    done = 0
    for n in checkpoints:
        for lt in lats.values():
            lt.step(n - done)
        done = n
        fr = {q: [round(float(v), 3) for v in lt.front()] for q, lt in lats.items()}
        out.append({"case": "rt_front", "W": W, "Re": Re, "n": n, "spike_bubble_z_q15": fr[15],
                    "spike_bubble_z_q19": fr[19]})
    for lt in lats.values():
        lt.destroy()
    return out


def throughput(q, W=256, steps=50):
    import torch
    w = _with_q(wl.rayleigh_taylor(W=W, Re=4000.0), q)
    lt = mplb.from_workload(w, "f32")
    lt.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lt.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lt.destroy()
    per = {15: 200, 19: 232}[q]
    return {"case": "throughput", "q": q, "W": W, "MLUPS": round(w.nodes * steps / dt / 1e6, 1),
            "ms_per_step": round(dt / steps * 1e3, 4), "algorithmic_bytes_per_lup": per,
            "algorithmic_TBps": round(per * w.nodes * steps / dt / 1e12, 3)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    args = ap.parse_args(argv)
    for q in (15, 19):
        for n, R in ((32, 8.0), (48, 12.0)):
            print(json.dumps(laplace_run(q, n=n, R=R, steps=args.steps)), flush=True)
    # the study switches on the D3Q15 model: finite differences on D3Q7, the
    # untruncated forcing
    for stencil, forcing in ((1, 0), (0, 1)):
        print(json.dumps(laplace_run(15, n=48, R=12.0, steps=args.steps, stencil=stencil, forcing=forcing)),
              flush=True)
    for row in front_run():
        print(json.dumps(row), flush=True)
    for q in (15, 19):
        print(json.dumps(throughput(q)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
