"""Field error of each storage precision against FP64 on the Rayleigh-Taylor
boxes (Sec. III C), with throughput and integral quantities.

All precisions of one box are resident together and advance in lockstep; at
each checkpoint every field is compared with the FP64 run as a relative L2
error (the FP64 GPU path itself matches the FP64 oracle to 1e-12 on boxes the
oracle can run).  One JSON line is printed per checkpoint and precision:

    python -m paper_1507_07294_amd.precision_study --W 128 --Re 256 \\
        --checkpoints 1000,3200,6400 --precisions f32,f16,bf16 [--q 19]

`--q 19` runs the D3Q19 variant of the Navier-Stokes lattice instead of the
paper's D3Q15.  `--sigma` replaces the printed surface tension (1e-4), with
which the step is linearly unstable in the bulk once the flow passes a few
thousandths (a Rayleigh-Taylor run diverges near t = 1); sigma = 1e-2 keeps
the bulk stable up to flow speeds of about 0.04, for runs beyond that time.

Integral quantities: total phi drift relative to sum |phi_0|, kinetic energy
(1/2) sum rho |u|^2, and the spike tip and bubble front (lowest and highest
zero crossing of phi along z).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import mplb
from . import workloads as wl

FIELDS = ("phi", "mu", "ux", "uy", "uz", "p")


def rel_l2(a, b):
    den = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / den if den > 0 else float(np.linalg.norm(a - b))


def kinetic_energy(lt):
    rho = lt.read("rho")
    e = 0.0
    for f in ("ux", "uy", "uz"):
        u = lt.read(f)
        e += float(np.sum(rho * u * u))
    return 0.5 * e


def run(W, Re, checkpoints, precisions, log=print, q=15, sigma=1e-4):
    import torch
    w = wl.rayleigh_taylor(W=W, Re=Re, sigma=sigma)
    w.nse_q = q  # lattice of the Navier-Stokes populations
    names = ["f64"] + [p for p in precisions if p != "f64"]
    lats = {p: mplb.from_workload(w, p) for p in names}
    for lt in lats.values():
        lt.set_check_interval(500)
    phi_abs = float(np.abs(w.phi0).sum())
    phi_tot0 = {p: lt.totals()[0] for p, lt in lats.items()}
    done = 0
    rows = []
    for n in checkpoints:
        prev = done
        secs = {}
        for p, lt in list(lats.items()):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                lt.step(n - done)
            except mplb.MplbError as e:  # a precision that diverges is reported and dropped
                log(json.dumps({"W": W, "Re": Re, "q": q, "sigma": sigma, "n": n, "precision": p, "diverged": str(e)}))
                if p == "f64":  # no reference left
                    for other in lats.values():
                        other.destroy()
                    return rows
                lt.destroy()
                del lats[p]
                continue
            torch.cuda.synchronize()
            secs[p] = time.perf_counter() - t0
        done = n
        ref = {f: lats["f64"].read(f) for f in FIELDS}
        for p, lt in lats.items():
            row = {"W": W, "Re": Re, "q": q, "sigma": sigma, "n": n, "precision": p,
                   "MLUPS_segment": round(w.nodes * (n - prev) / secs[p] / 1e6, 1)}
            if p != "f64":
                row["rel_l2_vs_f64"] = {f: float(f"{rel_l2(lt.read(f), ref[f]):.3e}") for f in FIELDS}
            tot = lt.totals()
            row["phi_drift"] = float(f"{(tot[0] - phi_tot0[p]) / phi_abs:.3e}")
            row["kinetic_energy"] = float(f"{kinetic_energy(lt):.6e}")
            row["spike_bubble_z"] = [round(float(v), 4) for v in lt.front()]
            log(json.dumps(row))
            rows.append(row)
        del ref
    for lt in lats.values():
        lt.destroy()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--W", type=int, default=128)
    ap.add_argument("--Re", type=float, default=256.0)
    ap.add_argument("--checkpoints", default="1000,3200,6400")
    ap.add_argument("--precisions", default="f32,f16,bf16")
    ap.add_argument("--q", type=int, default=15, choices=(15, 19), help="NSE lattice: D3Q15 or D3Q19")
    ap.add_argument("--sigma", type=float, default=1e-4, help="surface tension (printed: 1e-4)")
    args = ap.parse_args(argv)
    cps = [int(v) for v in args.checkpoints.split(",") if v]
    if cps != sorted(cps) or not cps or cps[0] < 1:
        ap.error("checkpoints must be increasing and positive")
    run(args.W, args.Re, cps, [p for p in args.precisions.split(",") if p],
        log=lambda s: print(s, flush=True), q=args.q, sigma=args.sigma)
    return 0


if __name__ == "__main__":
    sys.exit(main())
