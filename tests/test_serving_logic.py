"""Host logic of the serving loop with a stand-in backend (CPU only):
admission by budget, FIFO order, every request completes once, batching,
and read-out only after the chunk that finished a lattice."""
import contextlib
import types

import pytest

from paper_1507_07294_amd import serve
from paper_1507_07294_amd import workloads as wl


class FakeLattice:
    def __init__(self, req):
        self.req = req
        self.steps = 0
        self.alive = True

    def step(self, k):
        self.steps += k

    def read(self, f):
        return self.steps

    failed = False  # stands for a lattice whose non-finite flag is set

    def check_finite(self):
        return 5 if self.failed else 0

    def last_error(self):
        return "non-finite population after step %d" % self.steps

    def set_stream(self, ptr):
        self.stream = ptr

    def set_check_interval(self, k):
        self.check_interval = k

    def destroy(self):
        self.alive = False


class FakeStreams:
    """Events are the number of chunks enqueued when they were recorded."""
    chunks = 0
    waited = []

    def main_ptr(self):
        return 1

    def side_ptr(self):
        return 2

    def on_side(self):
        return contextlib.nullcontext()

    def mark_main(self):
        return FakeStreams.chunks

    def side_waits(self, ev):
        FakeStreams.waited.append(ev)


@pytest.fixture
def fake(monkeypatch):
    state = types.SimpleNamespace(live=0, peak=0, batches=[])

    def from_workload(w, precision):
        state.live += 1
        state.peak = max(state.peak, state.live)
        lt = FakeLattice(w)
        orig = lt.destroy

        def destroy():
            state.live -= 1
            orig()
        lt.destroy = destroy
        return lt

    def step_many(lts, k):
        state.batches.append(len(lts))
        FakeStreams.chunks += 1
        for lt in lts:
            assert lt.stream == 1  # batched steps on the main stream
            lt.step(k)

    monkeypatch.setattr(serve.mplb, "from_workload", from_workload)
    monkeypatch.setattr(serve.mplb, "mplb_step_many", step_many)
    monkeypatch.setattr(serve, "_required", lambda req, precision: req.workload.nodes * 100)
    monkeypatch.setattr(serve, "_Streams", FakeStreams)
    FakeStreams.chunks, FakeStreams.waited = 0, []
    return state


def _trace(n=12):
    out = []
    for i in range(n):
        w = wl.static_droplet(n=8 + 4 * (i % 3), R=2.0)
        out.append(wl.Request(i, 0.0, "droplet", w.shape, w, 10 + 7 * i))
    return out


def test_budget_limits_residency(fake):
    trace = _trace()
    budget = 3 * 16 ** 3 * 100  # three of the largest boxes
    srv = serve.Server("f32", budget, chunk=5, keep_fields=True)
    results, summary = srv.run(trace, realtime=False)
    assert srv.peak_bytes <= budget
    assert fake.live == 0
    assert sorted(r.rid for r in results) == list(range(len(trace)))
    for r in results:
        assert r.fields["phi"] == trace[r.rid].steps  # stepped exactly to its target
    assert max(fake.batches) > 1 and summary["requests"] == len(trace)
    # each read-out waited for a chunk that had been enqueued, and a later
    # chunk was enqueued before the read (the read overlaps it)
    assert len(FakeStreams.waited) == len(trace)
    assert all(1 <= ev <= FakeStreams.chunks for ev in FakeStreams.waited)


def test_request_over_budget_is_rejected(fake):
    trace = _trace(2)
    srv = serve.Server("f32", 10, chunk=5)
    with pytest.raises(ValueError):
        srv.run(trace, realtime=False)


def test_back_to_back_runs_one_at_a_time(fake):
    trace = _trace(5)
    results, summary = serve.run_back_to_back(trace, chunk=4, realtime=False, keep_fields=True)
    assert fake.peak == 1
    assert [r.rid for r in results] == list(range(5))
    assert all(r.fields["phi"] == trace[r.rid].steps for r in results)


def test_failed_request_is_retired_with_its_error(fake):
    """A lattice whose flag reports non-finite populations comes back with
    that error and no fields; the others are unaffected and every request
    still completes once."""
    trace = _trace(6)
    bad = {2, 4}

    def plant(req, lt):
        lt.failed = req.rid in bad

    srv = serve.Server("f32", 3 * 16 ** 3 * 100, chunk=5, keep_fields=True, on_admit=plant)
    results, summary = srv.run(trace, realtime=False)
    assert summary["failed"] == 2 and fake.live == 0
    assert sorted(r.rid for r in results) == list(range(6))
    for r in results:
        if r.rid in bad:
            assert r.code == 5 and r.fields is None and "non-finite" in r.error
        else:
            assert r.code == 0 and r.error is None and r.fields["phi"] == trace[r.rid].steps
