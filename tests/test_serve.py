"""Scheduler of the serving loop, driven on the CPU by an executor that runs the FP64 oracle on worker threads.
The GPU path of the same scheduler is tested in test_gpu_serve.py."""
import concurrent.futures
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from paper_2201_00094_amd.serve import FrameRequest, FrameResult, RequestTooLarge, Server


class OracleExecutor:
    """Fake device: each launch resolves the frame with the oracle on a worker thread; footprint is a simple
    function of the frame so tests can reason about admission."""

    def __init__(self, orc, workers=4, delay=0.0, fail_tag=None):
        self.orc = orc
        self.pool = ThreadPoolExecutor(workers)
        self.delay = delay
        self.fail_tag = fail_tag
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0

    def footprint(self, req):
        return req.pixels * 100 + req.count * 10

    def _run(self, req):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        try:
            if self.delay:
                time.sleep(self.delay)
            f = req.frags
            r = self.orc.resolve(req.width, req.height, req.rank, f.pixel, f.depth, f.alpha, f.rgb, bg=req.bg,
                                 want=("out",))
            return r["out"]
        finally:
            with self.lock:
                self.active -= 1

    def launch(self, req, slot):
        if self.fail_tag is not None and req.tag == self.fail_tag:
            raise RuntimeError("launch failed on purpose")
        return self.pool.submit(self._run, req)

    def done(self, h):
        return h.done()

    def finish(self, h):
        return FrameResult(out=h.result())


def _req(seed, w, h, rank=3, tag=None):
    f = synth.frame_c1(seed=seed, width=w, height=h, rank=rank, mean=4.0)
    return FrameRequest(w, h, rank, f, bg=(0.2, 0.2, 0.2), tag=tag)


def test_all_requests_complete_with_their_own_result(orc):
    ex = OracleExecutor(orc)
    srv = Server(ex, slots=3, budget_bytes=10 ** 9)
    reqs = [_req(s, 8 + s, 5 + (s % 3), tag=s) for s in range(12)]
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    for r, q in zip(res, reqs):
        assert r.tag == q.tag
        alone = orc.resolve(q.width, q.height, q.rank, q.frags.pixel, q.frags.depth, q.frags.alpha, q.frags.rgb,
                            bg=q.bg, want=("out",))["out"]
        np.testing.assert_array_equal(r.out, alone)
        assert r.t_submit <= r.t_admit <= r.t_done
    s = srv.stats.summary()
    assert s["completed"] == 12 and s["max_inflight"] <= 3 and ex.max_active <= 3


def test_budget_is_never_exceeded_and_big_requests_serialise(orc):
    ex = OracleExecutor(orc, delay=0.02)
    big = [_req(100 + i, 40, 30, tag="big%d" % i) for i in range(3)]
    fp = max(ex.footprint(r) for r in big)
    srv = Server(ex, slots=4, budget_bytes=int(fp * 1.5))
    futs = [srv.submit(r) for r in big]
    for f in futs:
        f.result(timeout=60)
    srv.close()
    assert srv.stats.max_inflight == 1
    assert srv.stats.max_bytes_inflight <= int(fp * 1.5)


def test_oversized_request_is_rejected(orc):
    ex = OracleExecutor(orc)
    srv = Server(ex, slots=2, budget_bytes=1000)
    fut = srv.submit(_req(1, 16, 16))
    with pytest.raises(RequestTooLarge):
        fut.result(timeout=10)
    srv.close()
    assert srv.stats.rejected == 1


def test_backfill_admits_small_requests_behind_a_blocked_one(orc):
    ex = OracleExecutor(orc, delay=0.05)
    a = _req(1, 40, 30, tag="a")
    blocked = _req(2, 40, 30, tag="blocked")
    smalls = [_req(10 + i, 4, 4, tag="s%d" % i) for i in range(3)]
    fa = ex.footprint(a)
    srv = Server(ex, slots=4, budget_bytes=int(fa * 1.6), max_bypass=8)
    futs = [srv.submit(a), srv.submit(blocked)] + [srv.submit(r) for r in smalls]
    res = {f.result(timeout=60).tag: f.result() for f in futs}
    srv.close()
    # the small requests started before the blocked big one (it had to wait for `a`)
    assert all(res["s%d" % i].t_admit < res["blocked"].t_admit for i in range(3))


def test_bypass_limit_stops_backfilling(orc):
    ex = OracleExecutor(orc, delay=0.03)
    a = _req(1, 40, 30, tag="a")
    blocked = _req(2, 40, 30, tag="blocked")
    smalls = [_req(10 + i, 4, 4, tag="s%d" % i) for i in range(6)]
    fa = ex.footprint(a)
    srv = Server(ex, slots=8, budget_bytes=int(fa * 1.6), max_bypass=2)
    futs = [srv.submit(a), srv.submit(blocked)] + [srv.submit(r) for r in smalls]
    res = {f.result(timeout=60).tag: f.result() for f in futs}
    srv.close()
    passed = sum(res["s%d" % i].t_admit < res["blocked"].t_admit for i in range(6))
    assert passed <= 2


def test_launch_failure_is_reported_and_releases_resources(orc):
    ex = OracleExecutor(orc, fail_tag="bad")
    srv = Server(ex, slots=1, budget_bytes=10 ** 9)
    f_bad = srv.submit(_req(1, 8, 8, tag="bad"))
    f_ok = srv.submit(_req(2, 8, 8, tag="ok"))
    with pytest.raises(RuntimeError):
        f_bad.result(timeout=30)
    assert f_ok.result(timeout=30).tag == "ok"
    srv.close()


class FinishFailsExecutor(OracleExecutor):
    """Completion raises for one tag, as a device error surfacing when a frame's results are collected would."""

    def __init__(self, orc, bad_tag, **kw):
        super().__init__(orc, **kw)
        self.bad_tag = bad_tag

    def launch(self, req, slot):
        return (req.tag, super().launch(req, slot))

    def done(self, h):
        return h[1].done()

    def finish(self, h):
        if h[0] == self.bad_tag:
            raise RuntimeError("completion failed on purpose")
        return FrameResult(out=h[1].result())


def test_completion_failure_is_reported_and_the_scheduler_keeps_serving(orc):
    ex = FinishFailsExecutor(orc, "bad")
    srv = Server(ex, slots=1, budget_bytes=10 ** 9)
    f_bad = srv.submit(_req(1, 8, 8, tag="bad"))
    f_ok = [srv.submit(_req(2 + i, 8, 8, tag="ok%d" % i)) for i in range(3)]
    with pytest.raises(RuntimeError, match="on purpose"):
        f_bad.result(timeout=30)
    assert [f.result(timeout=30).tag for f in f_ok] == ["ok0", "ok1", "ok2"]
    srv.drain(timeout=30)
    assert srv.stats.failed == 1 and srv.stats.completed == 3
    assert srv._bytes == 0 and sorted(srv._free_slots) == [0]
    srv.close()


def test_submit_after_close_is_refused(orc):
    srv = Server(OracleExecutor(orc), slots=1, budget_bytes=10 ** 9)
    srv.close()
    with pytest.raises(RuntimeError, match="closed"):
        srv.submit(_req(1, 8, 8))


def test_poisson_trace_generator():
    tr = synth.poisson_arrivals(3, 200, rate_hz=100.0)
    assert len(tr) == 200
    t = np.array([r["t"] for r in tr])
    assert (np.diff(t) > 0).all()
    assert 1.0 < t[-1] < 4.0  # about 2 s of arrivals at 100/s
    assert {r["rank"] for r in tr} == {3, 4} and {r["dtype"] for r in tr} == {"f32", "f16"}


def test_cancelled_request_is_never_launched(orc):
    ex = OracleExecutor(orc, delay=0.2)
    srv = Server(ex, slots=1, budget_bytes=10 ** 9)
    f_run = srv.submit(_req(1, 8, 8, tag="running"))
    time.sleep(0.05)  # the first request holds the only slot
    f_cancel = srv.submit(_req(2, 8, 8, tag="cancelled"))
    f_next = srv.submit(_req(3, 8, 8, tag="next"))
    assert f_cancel.cancel()
    assert f_run.result(timeout=30).tag == "running"
    assert f_next.result(timeout=30).tag == "next"
    srv.drain(timeout=30)
    srv.close()
    assert f_cancel.cancelled()
    assert srv.stats.cancelled == 1 and srv.stats.completed == 2
    # an admitted request can no longer be cancelled
    srv2 = Server(OracleExecutor(orc, delay=0.1), slots=1, budget_bytes=10 ** 9)
    f = srv2.submit(_req(4, 8, 8, tag="admitted"))
    t0 = time.time()
    while not f.running() and time.time() - t0 < 10:
        time.sleep(0.005)
    assert not f.cancel()
    assert f.result(timeout=30).tag == "admitted"
    srv2.close()


def test_admission_deadline_fails_a_request_still_queued(orc):
    from paper_2201_00094_amd.serve import RequestTimeout
    ex = OracleExecutor(orc, delay=0.3)
    srv = Server(ex, slots=1, budget_bytes=10 ** 9)
    f_run = srv.submit(_req(1, 8, 8, tag="running"))
    time.sleep(0.02)
    q = _req(2, 8, 8, tag="late")
    q.timeout = 0.05
    f_late = srv.submit(q)
    patient = _req(3, 8, 8, tag="patient")
    patient.timeout = 30.0
    f_patient = srv.submit(patient)
    with pytest.raises(RequestTimeout):
        f_late.result(timeout=30)
    assert f_run.result(timeout=30).tag == "running"
    assert f_patient.result(timeout=30).tag == "patient"
    srv.close()
    assert srv.stats.timed_out == 1 and srv.stats.completed == 2


class ResidentExecutor(OracleExecutor):
    """Fake device whose slots keep resident buffers (as the GPU executor's workspace and coefficient arrays do):
    a launch grows its slot to the request's need; trim releases an idle slot. Records the largest amount of
    memory held (resident + in flight) at any launch."""

    def __init__(self, orc, slots, need, **kw):
        super().__init__(orc, **kw)
        self.have = [0] * slots
        self.need = need          # tag -> resident bytes the request needs
        self.trimmed = []
        self.inflight = 0
        self.peak = 0

    def footprint(self, req):
        return 10

    def growth(self, slot, req):
        return max(0, self.need[req.tag] - (0 if slot is None else self.have[slot]))

    def resident_bytes(self):
        return sum(self.have)

    def trim(self, slot):
        self.trimmed.append(slot)
        self.have[slot] = 0

    def launch(self, req, slot):
        self.have[slot] = max(self.have[slot], self.need[req.tag])
        with self.lock:
            self.inflight += 1
            self.peak = max(self.peak, sum(self.have) + 10 * self.inflight)
        fut = super().launch(req, slot)
        fut.add_done_callback(lambda _: self._done())
        return fut

    def _done(self):
        with self.lock:
            self.inflight -= 1


def test_resident_slot_buffers_count_against_the_budget(orc):
    B = 1000
    need = {"a": 600, "b": 450, "c": 450, "big": 2000}
    ex = ResidentExecutor(orc, slots=2, need=need, delay=0.05)
    srv = Server(ex, slots=2, budget_bytes=B)
    # "a" leaves 600 bytes resident in its slot; "b" then reuses that slot, and "c" cannot take the other slot
    # (600 + 450 + in-flight bytes > 1000) until a slot with room is free
    fa = srv.submit(_req(1, 8, 8, tag="a"))
    fa.result(timeout=30)
    fb, fc = srv.submit(_req(2, 8, 8, tag="b")), srv.submit(_req(3, 8, 8, tag="c"))
    rb, rc = fb.result(timeout=30), fc.result(timeout=30)
    assert rc.t_admit >= rb.t_done - 1e-3 or rb.t_admit >= rc.t_done - 1e-3  # they did not overlap
    fbig = srv.submit(_req(4, 8, 8, tag="big"))
    with pytest.raises(RequestTooLarge):
        fbig.result(timeout=10)
    srv.close()
    assert ex.peak <= B and srv.stats.max_bytes_inflight <= B


def test_idle_slot_buffers_are_released_when_a_request_needs_the_room(orc):
    need = {"x": 700}
    ex = ResidentExecutor(orc, slots=2, need=need)
    ex.have = [600, 500]  # both slots idle, left large by earlier requests
    srv = Server(ex, slots=2, budget_bytes=1000)
    r = srv.submit(_req(1, 8, 8, tag="x")).result(timeout=30)
    srv.close()
    assert r.slot == 0 and ex.trimmed == [1] and ex.peak <= 1000


class GatedExecutor:
    """Fake device whose requests finish only when the test releases them; records the order of launches."""

    def __init__(self):
        self.launched = []
        self.gates = {}

    def footprint(self, req):
        return 1

    def launch(self, req, slot):
        ev = threading.Event()
        self.gates[req.tag] = ev
        self.launched.append(req.tag)
        return ev

    def done(self, h):
        return h.is_set()

    def finish(self, h):
        return FrameResult(out=None)


def _sized(tag, count):
    """A request whose only property that matters here is its fragment count."""
    class _F:
        pass
    f = _F()
    f.count = count
    return FrameRequest(8, 8, 3, f, tag=tag)


def _wait_launched(ex, n, timeout=10.0):
    t0 = time.perf_counter()
    while len(ex.launched) < n:
        assert time.perf_counter() - t0 < timeout, "launches: %r" % ex.launched
        time.sleep(0.001)


def test_shortest_first_admits_the_smallest_queued_request():
    ex = GatedExecutor()
    srv = Server(ex, slots=1, budget_bytes=10 ** 6, policy="sjf")
    futs = [srv.submit(_sized("first", 100))]
    _wait_launched(ex, 1)
    for tag, n in (("big", 900), ("mid", 500), ("small", 10), ("mid2", 500)):
        futs.append(srv.submit(_sized(tag, n)))
    time.sleep(0.01)
    for k, expect in enumerate(("small", "mid", "mid2", "big"), start=1):
        ex.gates[ex.launched[k - 1]].set()
        _wait_launched(ex, k + 1)
        assert ex.launched[k] == expect, ex.launched
    ex.gates[ex.launched[-1]].set()
    for f in futs:
        f.result(timeout=10)
    srv.close()


def test_shortest_first_does_not_starve_a_large_request():
    """Every admission of a younger, smaller request passes the large one over once; after max_bypass of them it
    goes next although smaller requests are still queued."""
    ex = GatedExecutor()
    srv = Server(ex, slots=1, budget_bytes=10 ** 6, policy="sjf", max_bypass=2)
    futs = [srv.submit(_sized("first", 1))]
    _wait_launched(ex, 1)
    futs.append(srv.submit(_sized("large", 1000)))
    futs += [srv.submit(_sized("s%d" % k, 10 + k)) for k in range(4)]
    time.sleep(0.01)
    for k in range(1, 6):
        ex.gates[ex.launched[k - 1]].set()
        _wait_launched(ex, k + 1)
    assert ex.launched[:4] == ["first", "s0", "s1", "large"], ex.launched
    ex.gates[ex.launched[-1]].set()
    for f in futs:
        f.result(timeout=10)
    srv.close()


def test_policy_must_be_known():
    with pytest.raises(ValueError):
        Server(GatedExecutor(), policy="lifo")


# -- executors that can block on a completion: the scheduler is woken by its per-slot waiting threads ---------------
NEVER_POLLS = 30.0  # a poll interval no test here could wait out: progress must come from the waiting threads


class BlockingOracleExecutor(OracleExecutor):
    def wait(self, h):
        concurrent.futures.wait([h])


class BlockingGatedExecutor(GatedExecutor):
    def wait(self, h):
        h.wait()


def test_blocking_executor_completes_every_request_without_polling(orc):
    ex = BlockingOracleExecutor(orc)
    srv = Server(ex, slots=3, budget_bytes=10 ** 9, poll_interval=NEVER_POLLS)
    reqs = [_req(s, 8 + s, 5 + (s % 3), tag=s) for s in range(12)]
    t0 = time.perf_counter()
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=20) for f in futs]
    assert time.perf_counter() - t0 < 20
    srv.close()
    for r, q in zip(res, reqs):
        assert r.tag == q.tag
        alone = orc.resolve(q.width, q.height, q.rank, q.frags.pixel, q.frags.depth, q.frags.alpha, q.frags.rgb,
                            bg=q.bg, want=("out",))["out"]
        np.testing.assert_array_equal(r.out, alone)
        assert r.t_submit <= r.t_admit <= r.t_done
    s = srv.stats.summary()
    assert s["completed"] == 12 and s["max_inflight"] <= 3 and ex.max_active <= 3


def test_blocking_executor_admits_the_next_request_when_one_completes():
    """One slot, shortest first: each release of the running request's gate wakes the scheduler, which launches the
    next request at once (well within a second, against a poll interval of 30 s)."""
    ex = BlockingGatedExecutor()
    srv = Server(ex, slots=1, budget_bytes=10 ** 6, policy="sjf", poll_interval=NEVER_POLLS)
    futs = [srv.submit(_sized("first", 100))]
    _wait_launched(ex, 1, timeout=2.0)
    for tag, n in (("big", 900), ("small", 10), ("mid", 500)):
        futs.append(srv.submit(_sized(tag, n)))
    time.sleep(0.01)
    for k, expect in enumerate(("small", "mid", "big"), start=1):
        t0 = time.perf_counter()
        ex.gates[ex.launched[k - 1]].set()
        _wait_launched(ex, k + 1, timeout=2.0)
        assert ex.launched[k] == expect, ex.launched
        assert time.perf_counter() - t0 < 1.0
    ex.gates[ex.launched[-1]].set()
    for f in futs:
        f.result(timeout=5)
    srv.close()
    assert srv.stats.completed == 4


def test_blocking_executor_keeps_admission_deadlines():
    from paper_2201_00094_amd.serve import RequestTimeout
    ex = BlockingGatedExecutor()
    srv = Server(ex, slots=1, budget_bytes=10 ** 6, poll_interval=NEVER_POLLS)
    f_run = srv.submit(_sized("running", 10))
    _wait_launched(ex, 1, timeout=2.0)
    late = _sized("late", 10)
    late.timeout = 0.05
    t0 = time.perf_counter()
    f_late = srv.submit(late)
    with pytest.raises(RequestTimeout):
        f_late.result(timeout=5)
    assert time.perf_counter() - t0 < 1.0
    ex.gates["running"].set()
    f_run.result(timeout=5)
    srv.close()
    assert srv.stats.timed_out == 1 and srv.stats.completed == 1 and ex.launched == ["running"]
