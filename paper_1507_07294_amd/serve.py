"""Continuous-batching serving loop for many independent simulations.

Requests (a workload and a step target) arrive over time.  The loop admits
them as slots while their device bytes fit an HBM budget, keeps every
admitted lattice resident, and advances all of them together: one batched
step kernel per time step covers every active lattice (``mplb_step_many``).
A lattice that reaches its target is read out (fields to the host) and freed,
which makes room for the next admissions.  Requests that arrive while others
are on the GPU join at the next chunk boundary.  A lattice whose populations
became non-finite is retired with that error in its own result (no fields);
the lattices batched with it are unaffected.

The back-to-back reference runs the same requests one at a time, in arrival
order, with the same chunking.

    python -m paper_1507_07294_amd.serve [--requests 256] [--steps 2000] [--rt-steps 400] [--budget-gb 16]
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import sys
import time
from typing import Dict, List, Optional

import numpy as np

from . import mplb
from . import workloads as wl

READ_FIELDS = ("phi", "ux", "uy", "uz", "p")


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    lups: int
    fields: Optional[Dict[str, np.ndarray]] = None
    error: Optional[str] = None  # set when the simulation failed (non-finite populations)
    code: int = 0                # MPLB_OK, or the mplb error code of the failure

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def _required(req, precision):
    nx, ny, nz = req.workload.shape
    return mplb.mplb_required_bytes(nx, ny, nz, mplb.PRECISIONS[precision], mplb.MPLB_COUPLED)


def _summary(results: List[Result], t_first: float, t_last: float):
    lat = np.array([r.latency for r in results])
    lups = sum(r.lups for r in results)
    span = max(t_last - t_first, 1e-9)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": span, "aggregate_MLUPS": lups / span / 1e6,
            "failed": sum(1 for r in results if r.code != 0)}


class _Streams:
    """The current stream, which runs the batched steps, and a second one for
    setting lattices up and reading them out."""

    def __init__(self):
        import torch
        self._torch = torch
        self.main = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()

    def main_ptr(self):
        return self.main.cuda_stream

    def side_ptr(self):
        return self.side.cuda_stream

    def on_side(self):
        return self._torch.cuda.stream(self.side)

    def mark_main(self):
        ev = self._torch.cuda.Event()
        ev.record(self.main)
        return ev

    def side_waits(self, ev):
        self.side.wait_event(ev)


class Server:
    """Admits requests by HBM budget and advances all resident lattices with
    batched steps, `chunk` steps at a time."""

    def __init__(self, precision="f32", budget_bytes=16e9, chunk=50, keep_fields=False, on_admit=None):
        self.precision = precision
        # on_admit(request, lattice): called once a lattice is set up (a test
        # hook, e.g. to plant a fault in one request)
        self.on_admit = on_admit
        self.budget = float(budget_bytes)
        self.chunk = int(chunk)
        self.keep_fields = keep_fields
        self.peak_bytes = 0
        self.batch_sizes: List[int] = []

    def run(self, trace, realtime=True):
        """Serve the trace.  The batched steps go to the current stream; new
        lattices are set up and finished ones read out on a second stream, so
        that both overlap the steps: a chunk is enqueued before the lattices
        that the previous chunk finished are read out, and those reads wait
        only for that previous chunk (an event)."""
        st = _Streams()
        t0 = time.perf_counter()
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        waiting = collections.deque()
        active = []  # [req, lattice, done, admitted, bytes]
        finished = []  # (entry, event after the chunk that finished it)
        used = 0
        results: List[Result] = []
        while pending or waiting or active or finished:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            while waiting:
                req = waiting[0]
                need = _required(req, self.precision)
                if need > self.budget:
                    raise ValueError(f"request {req.rid} needs {need} B, more than the budget")
                if used + need > self.budget:
                    break
                waiting.popleft()
                with st.on_side():  # memory, upload and init on the side stream
                    lt = mplb.from_workload(req.workload, self.precision)  # returns initialised
                # no synchronising checks inside the batched steps: each
                # lattice's flag is read once it has finished (below)
                lt.set_check_interval(0)
                if self.on_admit is not None:
                    self.on_admit(req, lt)
                lt.set_stream(st.main_ptr())
                used += need
                self.peak_bytes = max(self.peak_bytes, used)
                active.append([req, lt, 0, time.perf_counter() - t0, need])
            just_finished = []
            if active:
                k = min(self.chunk, min(a[0].steps - a[2] for a in active))
                mplb.mplb_step_many([a[1] for a in active], k)
                ev = st.mark_main()
                self.batch_sizes.append(len(active))
                still = []
                for a in active:
                    a[2] += k
                    (just_finished if a[2] >= a[0].steps else still).append(a)
                active = still
                just_finished = [(a, ev) for a in just_finished]
            # read out what the previous chunk finished while this one runs
            for a, ev in finished:
                st.side_waits(ev)
                a[1].set_stream(st.side_ptr())
                code = a[1].check_finite()  # this lattice's own flag; synchronises the side stream
                if code == mplb.MPLB_OK:
                    fields, err = {f: a[1].read(f) for f in READ_FIELDS}, None
                else:
                    fields, err = None, a[1].last_error()
                done = time.perf_counter() - t0
                results.append(Result(a[0].rid, a[0].arrival, a[3], done, a[0].workload.nodes * a[0].steps,
                                      fields if self.keep_fields else None, err, code))
                a[1].destroy()
                used -= a[4]
            finished = just_finished
            if not active and not finished and pending and not waiting:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
        t_last = max(r.completed for r in results)
        t_first = min(r.arrival for r in results)
        return results, _summary(results, t_first, t_last)


def run_back_to_back(trace, precision="f32", chunk=50, realtime=True, keep_fields=False):
    """The same requests one at a time in arrival order (each alone on the GPU)."""
    t0 = time.perf_counter()
    results = []
    for req in sorted(trace, key=lambda r: r.arrival):
        if realtime:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        start = time.perf_counter() - t0
        lt = mplb.from_workload(req.workload, precision)
        done = 0
        while done < req.steps:
            k = min(chunk, req.steps - done)
            lt.step(k)
            done += k
        code = lt.check_finite()
        fields, err = ({f: lt.read(f) for f in READ_FIELDS}, None) if code == mplb.MPLB_OK else (None, lt.last_error())
        end = time.perf_counter() - t0
        results.append(Result(req.rid, req.arrival, start, end, req.workload.nodes * req.steps,
                              fields if keep_fields else None, err, code))
        lt.destroy()
    t_last = max(r.completed for r in results)
    t_first = min(r.arrival for r in results)
    return results, _summary(results, t_first, t_last)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000, help="steps of each droplet request")
    ap.add_argument("--rt-steps", type=int, default=400, help="steps of each Rayleigh-Taylor request")
    ap.add_argument("--gap-ms", type=float, default=5.0, help="mean Poisson inter-arrival time")
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--precision", default="f32")
    args = ap.parse_args(argv)
    trace = wl.serving_trace(n_requests=args.requests, steps=args.steps, mean_gap_s=args.gap_ms / 1e3,
                             rt_steps=args.rt_steps)
    srv = Server(args.precision, args.budget_gb * 1e9, args.chunk)
    _, mix = srv.run(trace)
    _, b2b = run_back_to_back(trace, args.precision, args.chunk)
    print(json.dumps({"serving": mix, "back_to_back": b2b, "peak_bytes": srv.peak_bytes,
                      "mean_batch": float(np.mean(srv.batch_sizes))}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
