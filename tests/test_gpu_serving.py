"""Serving loop on the GPU: every result of a batched, budget-limited mix is
bitwise the same as the simulation run alone, and the budget holds."""
import numpy as np
import pytest

from paper_1507_07294_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _trace():
    reqs = []
    specs = [("droplet", 32, 90), ("rt", 32, 70), ("droplet", 48, 110), ("droplet", 32, 50),
             ("rt", 32, 130), ("droplet", 40, 60), ("rt", 24, 80), ("droplet", 32, 100)]
    for rid, (kind, n, steps) in enumerate(specs):
        if kind == "droplet":
            w = wl.static_droplet(n=n, R=n / 4, ratio=2.0 + rid)
        else:
            w = wl.rayleigh_taylor(W=n, Re=256.0)
        reqs.append(wl.Request(rid, 0.0, kind, w.shape, w, steps))
    return reqs


@pytest.mark.parametrize("precision", ["f32", "f16", "bf16"])
def test_mix_equals_alone_and_budget_holds(precision):
    from paper_1507_07294_amd import mplb
    from paper_1507_07294_amd.serve import Server
    print(f"\n[case] serving mix {precision}", flush=True)
    trace = _trace()
    sizes = [mplb.mplb_required_bytes(*r.workload.shape, mplb.PRECISIONS[precision], mplb.MPLB_COUPLED)
             for r in trace]
    budget = sorted(sizes)[-1] + sorted(sizes)[-2] + 1  # about two lattices at a time: admission waits
    srv = Server(precision, budget, chunk=40, keep_fields=True)
    results, summary = srv.run(trace, realtime=False)
    print(f"\n[serving] {summary} peak={srv.peak_bytes} budget={budget} batches={srv.batch_sizes}", flush=True)
    assert srv.peak_bytes <= budget
    assert max(srv.batch_sizes) >= 2  # requests really ran together
    assert len(results) == len(trace)
    for res in results:
        req = trace[res.rid]
        lt = mplb.from_workload(req.workload, precision)
        lt.step(req.steps)
        for f, v in res.fields.items():
            assert np.array_equal(v, lt.read(f)), (res.rid, f)
        lt.destroy()


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_step_many_mixed_walls_and_parity(precision):
    """Lattices at different step parities and with walls on x or y batch
    together correctly."""
    from paper_1507_07294_amd import mplb
    print(f"\n[case] step_many walls and parity {precision}", flush=True)
    ws = [wl.perturbed_case((20, 18, 16), (0, 0, 1), 91), wl.perturbed_case((17, 21, 15), (1, 0, 0), 92),
          wl.perturbed_case((33, 9, 12), (0, 1, 1), 93)]
    alone = []
    for i, w in enumerate(ws):
        g = mplb.from_workload(w, precision)
        g.step(13 + i)
        alone.append({k: g.read(k) for k in ("phi", "ux", "p")})
        g.destroy()
    mix = [mplb.from_workload(w, precision) for w in ws]
    mix[1].step(1)
    mix[2].step(2)
    mplb.mplb_step_many(mix, 13)
    for g, ref in zip(mix, alone):
        for k, v in ref.items():
            assert np.array_equal(g.read(k), v), k


def test_graph_chunks_equal_direct_launches():
    """A chunk replayed as a graph (built once, reused while the batch keeps
    its shape, with the table rewritten between calls) equals the same steps
    launched one by one, bitwise."""
    from paper_1507_07294_amd import mplb
    ws = [wl.perturbed_case((24, 20, 18), (0, 0, 1), 94), wl.perturbed_case((19, 23, 17), (0, 0, 0), 95)]
    out = {}
    for graphs in (False, True):
        mplb.mplb_set_step_many_graphs(graphs)
        try:
            mix = [mplb.from_workload(w, "f32") for w in ws]
            mix[0].step(1)  # different parities
            for k in (7, 7, 5, 7, 1):  # repeated shape: graph reuse; k = 1: direct launch
                mplb.mplb_step_many(mix, k)
            out[graphs] = [{f: g.read(f) for f in ("phi", "mu", "ux", "uz", "p")} for g in mix]
            assert [g.step_count for g in mix] == [28, 27]
            for g in mix:
                g.destroy()
        finally:
            mplb.mplb_set_step_many_graphs(True)
    for a, b in zip(out[False], out[True]):
        for f in a:
            assert np.array_equal(a[f], b[f]), f


def test_large_batch_equals_alone():
    """A batch whose step moves more than the last-level cache (two 128^3
    FP32 lattices, about 0.8 GB per step) takes the streaming-store path;
    results are still bitwise those of each lattice alone."""
    from paper_1507_07294_amd import mplb
    ws = [wl.static_droplet(n=128, R=30.0, ratio=3.0), wl.static_droplet(n=128, R=22.0, ratio=5.0)]
    alone = []
    for w in ws:
        g = mplb.from_workload(w, "f32")
        g.step(6)
        alone.append({k: g.read(k) for k in ("phi", "uz", "p")})
        g.destroy()
    mix = [mplb.from_workload(w, "f32") for w in ws]
    mplb.mplb_step_many(mix, 6)
    for g, ref in zip(mix, alone):
        for k, v in ref.items():
            assert np.array_equal(g.read(k), v), k
        g.destroy()


def test_step_many_with_untruncated_forcing():
    """Lattices with the Eq. 28 forcing are stepped one after another by
    step_many (the batched kernel carries the printed Eq. 32 only); results
    equal separate runs bitwise."""
    from paper_1507_07294_amd import mplb
    ws = [wl.perturbed_case((20, 18, 16), (0, 0, 1), 71), wl.perturbed_case((17, 21, 15), (0, 0, 0), 72)]
    for w in ws:
        w.params = w.params.replace(forcing=1)
    alone = []
    for w in ws:
        g = mplb.from_workload(w, "f32")
        g.step(9)
        alone.append({k: g.read(k) for k in ("phi", "ux", "p")})
        g.destroy()
    mix = [mplb.from_workload(w, "f32") for w in ws]
    mplb.mplb_step_many(mix, 9)
    for g, ref in zip(mix, alone):
        for k, v in ref.items():
            assert np.array_equal(g.read(k), v), k
        g.destroy()


def test_nan_in_one_lattice_stays_in_that_lattice():
    """A NaN planted in one lattice of a batch: the other lattices still equal
    their results alone, bitwise, and only the poisoned one reports a
    non-finite population."""
    from paper_1507_07294_amd import mplb
    print("\n[case] NaN isolation in step_many", flush=True)
    ws = [wl.perturbed_case(s, (0, 0, 1), 95 + i, coupled=True) for i, s in
          enumerate([(16, 14, 12), (20, 10, 18), (12, 12, 12)])]
    alone = []
    for w in ws:
        g = mplb.from_workload(w, "f32")
        g.step(9)
        alone.append({k: g.read(k) for k in ("phi", "ux", "p")})
        g.destroy()
    mix = [mplb.from_workload(w, "f32") for w in ws]
    mix[1].poke(1, 7, 3 + 20 * 5, float("nan"))
    mplb.mplb_step_many(mix, 9)
    for i in (0, 2):
        for k, v in alone[i].items():
            assert np.array_equal(mix[i].read(k), v), (i, k)
        rc, _ = mix[i].try_totals()
        assert rc == 0
    rc, _ = mix[1].try_totals()
    assert rc == mplb.MPLB_E_NONFINITE
    for g in mix:
        g.destroy()


@pytest.mark.parametrize("q19", [False, True])
def test_step_many_reports_every_failed_lattice(q19):
    """With a check interval set, step_many checks each lattice whose interval
    was crossed and names every failed one, not only the first; the others
    still equal their runs alone.  The D3Q19 batch takes the one-after-another
    path, which checks the same way."""
    from paper_1507_07294_amd import mplb
    print(f"\n[case] step_many per-lattice failures q19={q19}", flush=True)
    ws = [wl.perturbed_case(s, (0, 0, 1), 120 + i, coupled=True) for i, s in
          enumerate([(16, 14, 12), (20, 10, 18), (12, 12, 12), (14, 16, 10)])]
    for w in ws:
        w.nse_q = 19 if q19 else 15
    alone = []
    for w in ws:
        g = mplb.from_workload(w, "f32")
        g.step(10)
        alone.append({k: g.read(k) for k in ("phi", "uz")})
        g.destroy()
    mix = [mplb.from_workload(w, "f32") for w in ws]
    for g in mix:
        g.set_check_interval(5)
    mix[0].poke(1, 7, 40, float("nan"))
    mix[2].poke(0, 3, 11, float("inf"))
    with pytest.raises(mplb.NonFiniteError) as ei:
        mplb.mplb_step_many(mix, 10)
    assert ei.value.failed == [0, 2]
    assert all("non-finite" in m for m in ei.value.messages)
    for i in (1, 3):
        assert mix[i].check_finite() == mplb.MPLB_OK
        for k, v in alone[i].items():
            assert np.array_equal(mix[i].read(k), v), (i, k)
    for g in mix:
        g.destroy()


def test_served_request_that_fails_is_retired_alone():
    """A NaN planted in one served request: that request comes back with
    MPLB_E_NONFINITE and no fields; every other request's fields are bitwise
    its run alone."""
    from paper_1507_07294_amd import mplb
    from paper_1507_07294_amd.serve import Server
    print("\n[case] serving with one failing request", flush=True)
    trace = _trace()[:5]
    bad = 2

    def plant(req, lt):
        if req.rid == bad:
            lt.poke(1, 8, lt.N // 2, float("nan"))

    srv = Server("f32", 64e9, chunk=30, keep_fields=True, on_admit=plant)
    results, summary = srv.run(trace, realtime=False)
    assert summary["failed"] == 1
    assert max(srv.batch_sizes) >= 2
    for res in results:
        if res.rid == bad:
            assert res.code == mplb.MPLB_E_NONFINITE and res.fields is None and "non-finite" in res.error
            continue
        assert res.code == 0 and res.error is None
        req = trace[res.rid]
        lt = mplb.from_workload(req.workload, "f32")
        lt.step(req.steps)
        for f, v in res.fields.items():
            assert np.array_equal(v, lt.read(f)), (res.rid, f)
        lt.destroy()
