"""Serving loop logic on the CPU: a fake executor and a fake clock drive the
scheduler (admission by slots and HBM budget, FIFO order, same-library
batching, continuous admission, rejection, cancellation, failures)."""
import numpy as np
import pytest

from paper_2111_07347_amd.serve import BudgetError, Scheduler, Server, latency_report


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each batch takes `per_row` seconds per row (fake clock); results encode
    the request id so mix-ups are visible."""

    def __init__(self, clock, per_row=0.010, fail_libs=(), hang_libs=()):
        self.clock, self.per_row = clock, per_row
        self.fail_libs, self.hang_libs = set(fail_libs), set(hang_libs)
        self.running = {}
        self.launched = []

    def launch(self, b):
        if b.lib_id in self.fail_libs:
            raise RuntimeError("device error")
        dur = float("inf") if b.lib_id in self.hang_libs else self.per_row * len(b.requests)
        self.running[b.slot] = (self.clock() + dur, b)
        self.launched.append([r.req_id for r in b.requests])

    def done(self, slot):
        return slot in self.running and self.clock() >= self.running[slot][0]

    def collect(self, b):
        self.running.pop(b.slot)
        return [(np.full((r.n_patterns, 2), r.req_id, np.int32),
                 np.zeros((r.n_patterns, 2), np.int32),
                 np.full((r.n_patterns, 2), r.req_id, np.float32)) for r in b.requests]


def run(server, clock, until, dt=0.001):
    out = []
    while clock.t < until:
        out += server.step()
        clock.t += dt
    return out


def test_slot_limit_and_fifo():
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=10**9, slots=2, max_batch_rows=1, clock=clock)
    ids = [srv.submit(None, lib_id=i % 3, n_patterns=4, nbytes=100) for i in range(5)]
    srv.step()
    assert ex.launched == [[0], [1]]                 # two slots
    res = run(srv, clock, 0.1)
    assert [l[0] for l in ex.launched] == ids        # FIFO
    assert sorted(r.req_id for r in res) == ids
    for r in res:
        assert np.all(r.top_template == r.req_id)


def test_budget_admission_and_rejection():
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=1000, slots=4, max_batch_rows=4, clock=clock)
    for _ in range(3):
        srv.submit(None, lib_id=0, n_patterns=1, nbytes=600)   # only one fits at a time
    srv.step()
    assert len(srv.sched.inflight) == 1 and srv.sched.used == 600
    run(srv, clock, 0.05)
    assert srv.sched.idle and srv.sched.used == 0
    assert [len(l) for l in ex.launched] == [1, 1, 1]
    with pytest.raises(BudgetError):
        srv.submit(None, lib_id=0, n_patterns=1, nbytes=1001)
    with pytest.raises(ValueError):
        Scheduler(0, 1)


def test_same_library_batching_and_continuous_admission():
    clock = Clock()
    ex = FakeExecutor(clock, per_row=0.010)
    srv = Server(ex, budget_bytes=10**9, slots=1, max_batch_rows=3, clock=clock)
    srv.submit(None, 0, 2, 10)          # occupies the only slot
    srv.step()
    for lib in (1, 1, 2, 1, 1):         # arrive while the slot is busy
        srv.submit(None, lib, 2, 10)
    res = run(srv, clock, 0.2)
    # oldest queued (lib 1) first, joined by later lib-1 rows up to 3 rows;
    # the lib-2 row goes next, then the remaining lib-1 row
    assert ex.launched == [[0], [1, 2, 4], [3], [5]]
    assert len(res) == 6
    rep = latency_report(res)
    assert rep["rows"] == 6 and rep["p99_ms"] >= rep["p50_ms"] > 0
    assert rep["mean_batch_rows"] == pytest.approx((1 + 3 * 3 + 1 + 1) / 6)


def test_cancel_queued_request():
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=10**9, slots=1, max_batch_rows=1, clock=clock)
    a = srv.submit(None, 0, 1, 1)
    b = srv.submit(None, 0, 1, 1)
    srv.step()
    assert srv.sched.cancel(b) and not srv.sched.cancel(a)   # a is already running
    res = run(srv, clock, 0.05)
    assert [r.req_id for r in res] == [a]


def test_launch_failure_frees_slot_and_reports():
    clock = Clock()
    ex = FakeExecutor(clock, fail_libs=[7])
    srv = Server(ex, budget_bytes=10**9, slots=1, max_batch_rows=1, clock=clock)
    bad = srv.submit(None, 7, 1, 1)
    good = srv.submit(None, 0, 1, 1)
    res = run(srv, clock, 0.05)
    errs = {r.req_id: r.error for r in res}
    assert errs[bad].startswith("launch failed") and errs[good] is None
    assert srv.sched.idle


def test_watchdog_reports_hung_batch_once():
    clock = Clock()
    ex = FakeExecutor(clock, hang_libs=[3])
    srv = Server(ex, budget_bytes=10**9, slots=2, max_batch_rows=1, clock=clock, timeout_s=0.02)
    h = srv.submit(None, 3, 1, 1)
    ok = srv.submit(None, 0, 1, 1)
    res = run(srv, clock, 0.1)
    assert [r.error for r in res if r.req_id == h] == ["timeout"]
    assert [r.error for r in res if r.req_id == ok] == [None]
    assert len(srv.sched.inflight) == 1          # the hung slot stays occupied
    assert "p99_ms" in latency_report(res) and latency_report(res)["rows"] == 1
