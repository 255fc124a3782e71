"""The step kernel at the shape one GPU would hold if the 256 x 256 x 1024
Rayleigh-Taylor box were split into z-slabs over several GPUs.

The slab (nz / parts planes, through the interface) is periodic in z, which
stands in for the ghost planes a halo exchange would fill; the step itself
is the unchanged single-lattice step.  One JSON line per storage mode:

    python -m paper_1507_07294_amd.slab_study [--parts 8] [--steps 400]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

from . import mplb
from . import workloads as wl


def slab_run(parts=8, steps=400, precisions=("f32", "f16", "f64"), W=256):
    import torch
    big = wl.rayleigh_taylor(W=W, Re=4000.0)
    nz = big.shape[2] // parts
    z0 = big.shape[2] // 2 - nz // 2
    slab = dataclasses.replace(big, name=f"rt_slab_{W}x{W}x{nz}", shape=(W, W, nz), bc=(0, 0, 0),
                               phi0=big.phi0[z0:z0 + nz].copy())
    out = []
    for prec in precisions:
        lt = mplb.from_workload(slab, prec)
        lt.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out.append({"case": "slab", "shape": list(slab.shape), "parts": parts, "precision": prec,
                    "ms_per_step": round(dt * 1e3, 4), "GLUPS": round(slab.nodes / dt / 1e9, 2)})
        lt.destroy()
        del lt
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--parts", type=int, default=8)
    ap.add_argument("--steps", type=int, default=400)
    args = ap.parse_args(argv)
    for row in slab_run(args.parts, args.steps):
        print(json.dumps(row), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
