"""Flow speed along a Rayleigh-Taylor run (Sec. III C) until it diverges.

The D3Q7 step for the Cahn-Hilliard equation, linearised about a bulk phase
(phi = +-1, mu = 0) under a uniform flow u, is unstable at short wavelengths
once |u| exceeds a threshold that grows like the square root of the
mobility; with the printed surface tension (sigma = 1e-4) the bulk has almost
no diffusion of phi to damp it.  This study records, every few hundred steps,
the largest speed in the bulk (|phi| > 0.9) and overall, the range of phi and
whether the populations are still finite, so that the step at which the bulk
flow passes the threshold can be set beside the step at which the run fails:

    python -m paper_1507_07294_amd.stability_study --W 128 --Re 1024 --every 250 --steps 6000
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import mplb
from . import workloads as wl


def run(W, Re, steps, every, precision="f64", sigma=1e-4, log=print):
    w = wl.rayleigh_taylor(W=W, Re=Re, sigma=sigma)
    lt = mplb.from_workload(w, precision)
    lt.set_check_interval(0)  # the study reads the non-finite flag itself at each checkpoint
    rows = []
    n = 0
    while n < steps:
        k = min(every, steps - n)
        lt.step(k)
        n += k
        ok = lt.check_finite() == mplb.MPLB_OK
        row = {"W": W, "Re": Re, "sigma": sigma, "precision": precision, "n": n, "t": n * 0.04 / W,
               "finite": ok}
        if ok:
            phi = lt.read("phi")
            speed = np.sqrt(sum(lt.read(f) ** 2 for f in ("ux", "uy", "uz")))
            bulk = np.abs(phi) > 0.9
            row.update({"umax": float(speed.max()), "umax_bulk": float(speed[bulk].max()),
                        "phi_min": float(phi.min()), "phi_max": float(phi.max())})
        log(json.dumps(row))
        rows.append(row)
        if not ok:
            break
    lt.destroy()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--W", type=int, default=128)
    ap.add_argument("--Re", type=float, default=1024.0)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--precision", default="f64")
    ap.add_argument("--sigma", type=float, default=1e-4)
    args = ap.parse_args(argv)
    run(args.W, args.Re, args.steps, args.every, args.precision, args.sigma,
        log=lambda s: print(s, flush=True))
    return 0


if __name__ == "__main__":
    sys.exit(main())
