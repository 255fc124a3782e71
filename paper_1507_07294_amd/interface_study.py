"""Interface-capturing studies of the CHE-only step (Sec. III A-B).

* Zalesak's slotted sphere (Eq. 37) rotated for one revolution, MRT (S^f of
  Eq. 38) against SRT (every rate equal to s_1 of Eq. 38), over a range of
  Peclet numbers (Eq. 39, L = R).
* The deformation flow (Eq. 41) run for one period T, after which the
  interface returns to its start.

Both report the global relative error of Eq. 40 between phi at the end and
the initial field, the range of phi (an unstable run leaves [-1, 1] far
behind or diverges) and the throughput.  One JSON line per run:

    python -m paper_1507_07294_amd.interface_study [--precision f64] [--pe 200,400,600,800]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import mplb
from . import workloads as wl


def err_eq40(phi_end, phi_start):
    """Eq. 40: sum |phi(x, T) - phi(x, 0)| / sum |phi(x, 0)|."""
    phi_end = np.asarray(phi_end, dtype=np.float64)
    phi_start = np.asarray(phi_start, dtype=np.float64)
    return float(np.abs(phi_end - phi_start).sum() / np.abs(phi_start).sum())


def srt_rates(sf):
    """The SRT special case of an MRT rate set: every rate equal to s_1 (the
    rate that fixes the mobility through Eq. 19)."""
    return tuple([float(sf[1])] * 7)


def _run(w, precision, steps):
    import torch
    lt = mplb.from_workload(w, precision)
    lt.set_check_interval(1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = "ok"
    try:
        lt.step(steps)
        torch.cuda.synchronize()
    except mplb.MplbError as e:
        status = f"diverged: {e}"
    dt = time.perf_counter() - t0
    out = {"status": status, "MLUPS": round(w.nodes * steps / dt / 1e6, 1)}
    if status == "ok":
        phi = lt.read("phi")
        out.update({"Err": float(f"{err_eq40(phi, w.phi0):.4e}"), "phi_min": round(float(phi.min()), 4),
                    "phi_max": round(float(phi.max()), 4)})
    lt.destroy()
    return out


def zalesak_run(Pe, model="mrt", precision="f64", n=100, revolutions=1):
    """One revolution (10^4 steps at n = 100, U = 0.02) of Zalesak's sphere."""
    scale = n / 100.0
    w = wl.zalesak(n=n, R=40.0 * scale, slot=16.0 * scale, Pe=Pe)
    if model == "srt":
        w.params = dataclasses.replace(w.params, s_f=srt_rates(w.params.s_f))
    U = w.velocity["U"]
    steps = int(round(revolutions * 2 * n / U))  # period 2 pi / (U pi / n)
    return {"case": "zalesak", "n": n, "Pe": Pe, "model": model, "precision": precision, "steps": steps,
            **_run(w, precision, steps)}


def deformation_run(n=128, Pe=400.0, model="mrt", precision="f64", U=0.02, T=3.0):
    """One period of the deformation flow: t = n_steps U / n reaches T."""
    w = wl.deformation_flow(n=n, U=U, T=T, Pe=Pe)
    if model == "srt":
        w.params = dataclasses.replace(w.params, s_f=srt_rates(w.params.s_f))
    steps = int(round(T * n / U))
    return {"case": "deformation", "n": n, "Pe": Pe, "model": model, "precision": precision, "steps": steps,
            **_run(w, precision, steps)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="f64")
    ap.add_argument("--pe", default="200,400,600,800,1000")
    ap.add_argument("--deformation-n", default="64,128")
    args = ap.parse_args(argv)
    for Pe in [float(v) for v in args.pe.split(",") if v]:
        for model in ("mrt", "srt"):
            print(json.dumps(zalesak_run(Pe, model, args.precision)), flush=True)
    for n in [int(v) for v in args.deformation_n.split(",") if v]:
        for model in ("mrt", "srt"):
            print(json.dumps(deformation_run(n, 400.0, model, args.precision)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
