#!/usr/bin/env python3
"""Throughput of the MRT lattice-Boltzmann phase-field step on one MI355X.

Headline: the coupled step (D3Q7 Cahn-Hilliard + D3Q15 Navier-Stokes, surface
tension, gravity, bounce-back walls) on the 256 x 256 x 1024 Rayleigh-Taylor
box at Re = 4000, FP32 compute and storage, inputs resident in HBM.  Prints
one JSON line with MLUPS, the roofline of the dominant kernel (event-timed on
the library's stream), the storage-precision variants, the CHE-only
interface-tracking step, and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
# algorithmic bytes per lattice update (22 populations + 3-word (phi u)
# history, each read and written once), per storage mode
ALGO_BYTES = {"f64": 400, "f32": 200, "f16": 116, "bf16": 116}
Q19_ALGO_BYTES = {"f64": 464, "f32": 232, "f16": 132, "bf16": 132}  # D3Q19: 19 g instead of 15
CHE_ALGO_BYTES = {"f64": 2 * 8 * 8, "f32": 2 * 4 * 8}  # 7 populations + phi of the previous level


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--W", type=int, default=256, help="Rayleigh-Taylor box width (box W x W x 4W)")
    ap.add_argument("--variants", default="f16,bf16,f64", help="extra storage precisions to time ('' for none)")
    ap.add_argument("--no-che", action="store_true", help="skip the CHE-only interface-tracking line")
    ap.add_argument("--no-q19", action="store_true", help="skip the D3Q19 variant of the NSE lattice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain device copy of known size")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests in the serving trace (0: skip the serving leg)")
    ap.add_argument("--serving-steps", type=int, default=2000, help="steps of each droplet request")
    ap.add_argument("--serving-rt-steps", type=int, default=400,
                    help="steps of each Rayleigh-Taylor request (the printed parameters leave the physical "
                         "range near step 1000 on a W = 32 box and fail near 1800)")
    return ap.parse_args()


def _code_of(text):
    """C++ source without its comments and with runs of blank space folded:
    an edit of a comment is not a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(read=None):
    """Hash of the code of the step kernel's sources; a traffic figure taken on
    other code is not reported.  `read(name)` returns a source's text (default:
    the file in the package)."""
    if read is None:
        def read(name):
            with open(os.path.join(ROOT, "paper_1507_07294_amd", "csrc", name), encoding="utf-8") as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in ("fused.hip", "device.h", "common.h"):
        h.update(_code_of(read(f)).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = data.get(f"{kernel}|{workload}|{precision}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_lattice(lt, steps, warmup):
    import torch
    lt.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lt.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = lt.time_stages(max(1, min(steps, 50)))
    n_st = max(1, min(steps, 50))
    return dt, [v / n_st for v in stages]


def cpu_baseline(W, target_s=12.0, single_s=6.0):
    """The FP64 oracle on z-slabs of the same Rayleigh-Taylor box: on every
    host core (target_s of stepping), then on one thread (single_s, a thinner
    slab)."""
    import oracle.orc as orc
    from paper_1507_07294_amd import workloads as wl
    w = wl.rayleigh_taylor(W=W, Re=4000.0)

    def sample(nz_slab, budget_s):
        z0 = w.shape[2] // 2 - nz_slab // 2
        phi = w.phi0[z0:z0 + nz_slab].copy()
        shape = (w.shape[0], w.shape[1], nz_slab)
        o = orc.Oracle(shape, w.bc, orc.COUPLED, w.params)
        o.init(phi)
        # whole steps until budget_s of stepping has passed (at most 200 steps)
        steps, elapsed = 0, 0.0
        while elapsed < budget_s and steps < 200:
            t0 = time.perf_counter()
            o.step(1)
            elapsed += time.perf_counter() - t0
            steps += 1
        nodes = shape[0] * shape[1] * shape[2]
        return nodes * steps / elapsed / 1e6, steps, elapsed, f"{shape[0]}x{shape[1]}x{nz_slab}"

    cores = orc.threads()
    mlups, steps, secs, dims = sample(max(8, W // 2), target_s)
    orc.set_threads(1)
    try:
        m1, s1, t1, d1 = sample(max(4, W // 32), single_s)
    finally:
        orc.set_threads(cores)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "host": {"cpu_model": model, "nproc": os.cpu_count()},
            "sample": f"{dims} z-slab through the interface of the W={W} Rayleigh-Taylor box, "
                      f"{steps} FP64 steps, {secs:.1f} s",
            "single_thread": {"value": round(m1, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"{d1} z-slab, {s1} FP64 steps, {t1:.1f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a lattice larger than one "
              "GPU would be split into z-slabs with a halo exchange, which the library does not implement.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1507_07294_amd import mplb
    from paper_1507_07294_amd import workloads as wl

    W = args.W
    w = wl.rayleigh_taylor(W=W, Re=4000.0)
    N = w.nodes
    wname = f"rayleigh_taylor_{W}x{W}x{4 * W}_Re4000"
    print(f"[bench] {wname} N={N} f32: init", file=sys.stderr, flush=True)
    lt = mplb.from_workload(w, "f32")
    dt, st = time_lattice(lt, args.steps, args.warmup)
    # after the timed region: five more windows of steps/5 steps, for the
    # spread between windows (the median is reported beside the value)
    win = []
    for _ in range(5):
        k = max(1, args.steps // 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt.step(k)
        torch.cuda.synchronize()
        win.append((time.perf_counter() - t0) / k * 1e3)
    mlups = N * args.steps / dt / 1e6
    ms_step = dt / args.steps * 1e3
    k_ms = st[2]
    achieved = ALGO_BYTES["f32"] * N / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic("k_fused", wname, "f32")
    result = {
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wname, "nodes": N, "precision": "f32 compute and storage",
                   "boundaries": "periodic x,y; bounce-back walls z", "Re": 4000, "atwood": 0.5},
        "hbm_frac_step": round(ALGO_BYTES["f32"] * N / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "algorithmic_bytes_per_lup": ALGO_BYTES["f32"],
        "stage_ms": {"step": round(st[2], 4)},
        "windows_ms_per_step": [round(v, 4) for v in win],
        "median_window_ms_per_step": round(sorted(win)[2], 4),
        "roofline": {"kernel": "k_fused", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": ALGO_BYTES["f32"] * N},
    }
    lt.destroy()
    del lt
    torch.cuda.empty_cache()

    variants = {}
    for prec in [v for v in args.variants.split(",") if v]:
        print(f"[bench] {wname} {prec}", file=sys.stderr, flush=True)
        lt = mplb.from_workload(w, prec)
        steps = max(10, args.steps // (2 if prec == "f64" else 1))
        dtv, stv = time_lattice(lt, steps, max(2, args.warmup // 2))
        mv = N * steps / dtv / 1e6
        variants[prec] = {"MLUPS": round(mv, 1), "ms_per_step": round(dtv / steps * 1e3, 4),
                          "algorithmic_bytes_per_lup": ALGO_BYTES[prec],
                          "hbm_frac_step": round(ALGO_BYTES[prec] * N / (dtv / steps) / 1e9 / HBM_PEAK_GBPS, 4),
                          "k_step_ms": round(stv[2], 4)}
        lt.destroy()
        del lt
        torch.cuda.empty_cache()
    if variants:
        result["variants"] = variants

    if not args.no_q19:
        for prec in ("f32", "f16"):
            print(f"[bench] {wname} {prec} D3Q19", file=sys.stderr, flush=True)
            w.nse_q = 19
            lt = mplb.from_workload(w, prec)
            w.nse_q = 15
            steps = max(10, args.steps // 2)
            dtq, stq = time_lattice(lt, steps, max(2, args.warmup // 2))
            rec = {"MLUPS": round(N * steps / dtq / 1e6, 1), "ms_per_step": round(dtq / steps * 1e3, 4),
                   "algorithmic_bytes_per_lup": Q19_ALGO_BYTES[prec],
                   "hbm_frac_step": round(Q19_ALGO_BYTES[prec] * N / (dtq / steps) / 1e9 / HBM_PEAK_GBPS, 4),
                   "k_step_ms": round(stq[2], 4)}
            result["d3q19" if prec == "f32" else f"d3q19_{prec}"] = rec
            lt.destroy()
            del lt
            torch.cuda.empty_cache()

    if not args.no_che:
        # the interface-tracking step on the 128^3 box of the paper's tests
        # (its 126 MB stay in the last-level cache) and on 256^3 (1.07 GB
        # moved per step, bound by HBM)
        for n, key in ((128, "che_only"), (256, "che_only_256")):
            wc = wl.deformation_flow(n=n)
            print(f"[bench] deformation_flow {n}^3 f32 (CHE only)", file=sys.stderr, flush=True)
            lt = mplb.from_workload(wc, "f32")
            steps = args.steps
            dtc, stc = time_lattice(lt, steps, args.warmup)
            kc = CHE_ALGO_BYTES["f32"] * wc.nodes / (stc[2] * 1e-3) / 1e9
            result[key] = {"workload": f"deformation_flow_{n}^3", "MLUPS": round(wc.nodes * steps / dtc / 1e6, 1),
                           "ms_per_step": round(dtc / steps * 1e3, 4),
                           "algorithmic_bytes_per_lup": CHE_ALGO_BYTES["f32"],
                           "hbm_frac_step": round(CHE_ALGO_BYTES["f32"] * wc.nodes / (dtc / steps) / 1e9
                                                  / HBM_PEAK_GBPS, 4),
                           "k_step_ms": round(stc[2], 4), "k_achieved_GBps": round(kc, 1),
                           "k_frac": round(kc / HBM_PEAK_GBPS, 4),
                           "kernel": "k_fused_che2" if n >= 256 else "k_fused_che",
                           "traffic": measured_traffic("k_fused_che2" if n >= 256 else "k_fused_che",
                                                       f"deformation_flow_{n}^3", "f32")}
            lt.destroy()
            del lt
            torch.cuda.empty_cache()
        # the same 256^3 step with 16-bit storage of f_1..f_6 (f_0 and phi of
        # the previous level FP32): 40 B per update
        wc = wl.deformation_flow(n=256)
        lt = mplb.from_workload(wc, "f16")
        dtc, stc = time_lattice(lt, args.steps, args.warmup)
        result["che_only_256_f16"] = {"workload": "deformation_flow_256^3", "kernel": "k_fused_che2",
                                      "MLUPS": round(wc.nodes * args.steps / dtc / 1e6, 1),
                                      "ms_per_step": round(dtc / args.steps * 1e3, 4), "algorithmic_bytes_per_lup": 40,
                                      "k_step_ms": round(stc[2], 4),
                                      "k_frac": round(40 * wc.nodes / (stc[2] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                      "traffic": measured_traffic("k_fused_che2", "deformation_flow_256^3", "f16")}
        lt.destroy()
        del lt
        torch.cuda.empty_cache()

    if args.copy_probe:
        # bandwidth reference: the library's 16-byte copies (plain, streaming
        # stores, and four elements per thread with streaming loads and
        # stores) and the runtime's own device copy, each over 4 GiB
        nbytes = 4 << 30
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        probe = {}
        for name, fn in (("mplb_copy_probe", lambda: mplb.mplb_copy_probe(a, b, nbytes)),
                         ("mplb_copy_probe_streaming", lambda: mplb.mplb_copy_probe(a, b, nbytes, 1)),
                         ("mplb_copy_probe_x4", lambda: mplb.mplb_copy_probe(a, b, nbytes, 2)),
                         ("mplb_copy_probe_chunk256k", lambda: mplb.mplb_copy_probe(a, b, nbytes, 3)),
                         ("torch_copy", lambda: b.copy_(a))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
            probe[name] = round(2 * nbytes / ((time.perf_counter() - t0) / 10) / 1e9, 1)
        result["copy_probe_GBps"] = probe
        del a, b
        torch.cuda.empty_cache()

    if args.serving_requests > 0:
        from paper_1507_07294_amd import serve
        print(f"[bench] serving {args.serving_requests} requests x {args.serving_steps} / {args.serving_rt_steps} "
              "steps", file=sys.stderr, flush=True)
        trace = wl.serving_trace(n_requests=args.serving_requests, steps=args.serving_steps, mean_gap_s=0.003,
                                 rt_steps=args.serving_rt_steps)
        srv = serve.Server("f32", 16e9, chunk=50)
        _, mix = srv.run(trace)
        mplb.mplb_set_step_many_graphs(False)  # the same batched loop, steps launched one by one
        try:
            _, mix_nog = serve.Server("f32", 16e9, chunk=50).run(trace)
        finally:
            mplb.mplb_set_step_many_graphs(True)
        _, b2b = serve.run_back_to_back(trace, "f32", chunk=50)
        # the same trace with FP16 population storage (its field error against
        # the FP64 oracle is stated by the parity tests: 5e-3 relative L2)
        srv16 = serve.Server("f16", 16e9, chunk=50)
        _, mix16 = srv16.run(trace)
        result["serving"] = {
            "trace": f"{args.serving_requests} requests, Poisson arrivals (mean gap 3 ms, seed 20261202), half "
                     f"droplets (32^3..128^3, {args.serving_steps} steps each) half Rayleigh-Taylor (W = 32..64, "
                     f"{args.serving_rt_steps} steps each: the printed parameters leave the physical range near "
                     "step 1000 at W = 32), FP32, HBM budget 16 GB",
            "batched": {k: round(v, 4) for k, v in mix.items()},
            "batched_without_graphs": {k: round(v, 4) for k, v in mix_nog.items()},
            "back_to_back": {k: round(v, 4) for k, v in b2b.items()},
            "batched_f16_storage": {k: round(v, 4) for k, v in mix16.items()},
            "mean_batch": round(float(sum(srv.batch_sizes) / max(1, len(srv.batch_sizes))), 2),
            "peak_bytes": srv.peak_bytes}

    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
