"""Continuous-batching server for wavelet resolves.

Frames of different sizes, ranks and coefficient storage types arrive as requests. The scheduler admits a request
as soon as an execution slot is free and its HBM footprint fits the remaining budget, launches it on that slot's
HIP stream, and learns of completions by polling the executor (or, for an executor that can block on a
request's completion, from one waiting thread per slot that wakes the scheduler): requests that arrive while
others run are admitted as slots and memory free up, and their work overlaps on the GPU. Per-slot buffers
(workspace and coefficient array) stay resident and are reused across requests; the budget counts them as well
as the requests in flight. Latency is measured from arrival (submit) to the moment the completion event is
observed.

A queued request can be cancelled (``Future.cancel()``, until it is admitted) or given an admission deadline
(``FrameRequest.timeout``: seconds from submit; a request still queued then fails with :class:`RequestTimeout`).
Work already launched on the GPU runs to completion.

The scheduler is independent of the device: it drives an executor with ``footprint``, ``launch``, ``done`` and
``finish``, and optionally ``prepare`` (called on the submitting thread; its token is passed to ``launch``),
``wait`` (blocks until a launched request's work is complete; without it the scheduler polls ``done``) and
``growth`` / ``resident_bytes`` / ``trim`` (resident per-slot buffers). :class:`GpuExecutor` runs the library;
tests drive the scheduler with CPU executors.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class FrameRequest:
    width: int
    height: int
    rank: int
    frags: object                 # paper_2201_00094_amd.Fragments (device tensors)
    dtype: str = "f32"
    channels: int = 1
    bg: tuple = (0.0, 0.0, 0.0)
    want_coeffs: bool = False
    tag: object = None
    timeout: float = None         # admission deadline in seconds from submit (None: wait as long as it takes)
    out: object = None            # optional [P, 3] float32 device tensor the composite is written to (else allocated)

    @property
    def pixels(self) -> int:
        return self.width * self.height

    @property
    def count(self) -> int:
        return self.frags.count


@dataclass
class FrameResult:
    out: object                   # [P, 3] float32 (device tensor for the GPU executor)
    coeffs: object = None
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    tag: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class RequestTooLarge(RuntimeError):
    pass


class RequestTimeout(TimeoutError):
    pass


@dataclass
class _Pending:
    req: FrameRequest
    fut: Future
    t_submit: float
    footprint: int
    token: object = None
    bypassed: int = 0


@dataclass
class _Running:
    pend: _Pending
    slot: int
    handle: object
    t_admit: float


@dataclass
class ServerStats:
    completed: int = 0
    rejected: int = 0
    failed: int = 0      # launch or completion raised; reported on the request's future
    cancelled: int = 0   # cancelled by the client while queued
    timed_out: int = 0   # still queued at their admission deadline
    fragments: int = 0
    latencies: list = field(default_factory=list)
    waits: list = field(default_factory=list)   # arrival to admission
    max_inflight: int = 0
    max_bytes_inflight: int = 0
    first_submit: float = float("inf")
    last_done: float = 0.0

    def summary(self) -> dict:
        lat = np.array(self.latencies) * 1e3 if self.latencies else np.zeros(1)
        span = max(self.last_done - self.first_submit, 1e-12)
        wait = np.array(self.waits) * 1e3 if self.waits else np.zeros(1)
        return {"completed": self.completed, "rejected": self.rejected, "failed": self.failed,
                "cancelled": self.cancelled, "timed_out": self.timed_out, "fragments": self.fragments,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "fragments_per_s": self.fragments / span,
                "queued": int((wait > 1.0).sum()), "wait_p50_ms": float(np.percentile(wait, 50)),
                "wait_p99_ms": float(np.percentile(wait, 99)),
                "max_inflight": self.max_inflight, "max_bytes_inflight": self.max_bytes_inflight}


class Server:
    """Admission by HBM footprint and free slots. ``policy="fifo"``: first come, first admitted, with bounded
    back-filling (a request that does not fit may be passed by later, smaller ones at most ``max_bypass`` times,
    after which admission waits for it). ``policy="sjf"``: the queued request with the fewest fragments that fits
    goes first, and a request passed over ``max_bypass`` times goes before any other (so none waits forever).

    The budget holds the footprints of the requests in flight plus the executor's resident per-slot buffers
    (``resident_bytes``), including what a slot's buffers must grow by to take the request (``growth``). When a
    request does not fit, the buffers of idle slots are released (``trim``) before it is left waiting."""

    def __init__(self, executor, slots: int = 3, budget_bytes: int = 96 << 30, max_bypass: int = 8,
                 poll_interval: float = 0.0002, clock=time.perf_counter, policy: str = "fifo"):
        if policy not in ("fifo", "sjf"):
            raise ValueError("policy must be 'fifo' or 'sjf'")
        self.policy = policy
        self.ex = executor
        self.slots = int(slots)
        self.budget = int(budget_bytes)
        self.max_bypass = int(max_bypass)
        self.poll_interval = poll_interval
        self.clock = clock
        self.stats = ServerStats()
        self._queue = collections.deque()
        self._running: list[_Running] = []
        self._free_slots = list(range(self.slots))
        self._bytes = 0
        self._prep = hasattr(executor, "prepare")
        self._cv = threading.Condition()
        self._stop = False
        # an executor that can block on a request's completion gets one waiting thread per slot, which wakes the
        # scheduler when the request it waits for is complete; otherwise the scheduler polls every poll_interval
        self._blocking = callable(getattr(executor, "wait", None))
        self._wq = [queue.SimpleQueue() for _ in range(self.slots)] if self._blocking else []
        for k, q in enumerate(self._wq):
            threading.Thread(target=self._wait_loop, args=(q,), name="wt-serve-wait-%d" % k, daemon=True).start()
        self._thread = threading.Thread(target=self._loop, name="wt-serve", daemon=True)
        self._thread.start()

    # -- client side --------------------------------------------------------------------------------------
    def submit(self, req: FrameRequest) -> Future:
        """Queue a request; the future resolves to its :class:`FrameResult`. The executor's ``prepare`` runs here,
        on the submitting thread (the GPU executor orders the request after the work this thread's current stream
        has queued on its inputs)."""
        fut: Future = Future()
        t = self.clock()
        fp = int(self.ex.footprint(req))
        fresh = int(self._growth(None, req))
        with self._cv:
            if self._stop:
                raise RuntimeError("the server is closed")
            self.stats.first_submit = min(self.stats.first_submit, t)
            if fp + fresh > self.budget:
                self.stats.rejected += 1
                fut.set_exception(RequestTooLarge("request needs %d bytes, the budget is %d" % (fp + fresh,
                                                                                                self.budget)))
                return fut
        token = self.ex.prepare(req) if self._prep else None
        with self._cv:
            if self._stop:
                raise RuntimeError("the server is closed")
            self._queue.append(_Pending(req, fut, t, fp, token))
            self._cv.notify()
        return fut

    def close(self, wait: bool = True):
        with self._cv:
            self._stop = True
            self._cv.notify()
        if wait:
            self._thread.join()

    def drain(self, timeout: float = None):
        """Block until every submitted request has finished."""
        t0 = time.perf_counter()
        while True:
            with self._cv:
                if not self._queue and not self._running:
                    return
            if timeout is not None and time.perf_counter() - t0 > timeout:
                raise TimeoutError("requests still pending")
            time.sleep(self.poll_interval)

    # -- scheduler ----------------------------------------------------------------------------------------
    def _growth(self, slot, req) -> int:
        g = getattr(self.ex, "growth", None)
        return int(g(slot, req)) if g else 0

    def _resident(self) -> int:
        r = getattr(self.ex, "resident_bytes", None)
        return int(r()) if r else 0

    def _held(self) -> int:
        return self._bytes + self._resident()

    def _fit_slot(self, p):
        """A free slot that can take p within the budget (the one whose buffers grow least), or None. Releases the
        buffers of other idle slots when that makes the request fit."""
        slot = min(self._free_slots, key=lambda k: self._growth(k, p.req))
        need = p.footprint + self._growth(slot, p.req)
        if self._held() + need <= self.budget:
            return slot
        trim = getattr(self.ex, "trim", None)
        if trim is not None:
            for k in self._free_slots:
                if k != slot:
                    trim(k)
            need = p.footprint + self._growth(slot, p.req)
            if self._held() + need <= self.budget:
                return slot
        return None

    def _drop_expired_locked(self):
        now = self.clock()
        keep = collections.deque()
        for p in self._queue:
            if p.fut.cancelled():
                self.stats.cancelled += 1
            elif p.req.timeout is not None and now - p.t_submit > p.req.timeout:
                self.stats.timed_out += 1
                p.fut.set_exception(RequestTimeout("request still queued %.3f s after submit (timeout %.3f s)" %
                                                   (now - p.t_submit, p.req.timeout)))
            else:
                keep.append(p)
        self._queue = keep

    def _start_locked(self, i, slot):
        """Launch queue[i] on slot (or drop it if its client cancelled it meanwhile); on success every request
        ahead of it in the queue has been passed over once more."""
        p = self._queue[i]
        del self._queue[i]
        if not p.fut.set_running_or_notify_cancel():  # cancelled by the client meanwhile
            self.stats.cancelled += 1
            return
        self._free_slots.remove(slot)
        self._bytes += p.footprint
        t = self.clock()
        try:
            handle = self.ex.launch(p.req, slot, p.token) if self._prep else self.ex.launch(p.req, slot)
        except Exception as e:  # launch failure: report to the client, release resources
            self._bytes -= p.footprint
            self._free_slots.append(slot)
            self.stats.failed += 1
            p.fut.set_exception(e)
            return
        self._running.append(_Running(p, slot, handle, t))
        if self._blocking:
            self._wq[slot].put(handle)
        self.stats.max_inflight = max(self.stats.max_inflight, len(self._running))
        self.stats.max_bytes_inflight = max(self.stats.max_bytes_inflight, self._held())
        for q in list(self._queue)[:i]:
            q.bypassed += 1

    def _admit_locked(self):
        self._drop_expired_locked()
        if self.policy == "sjf":
            self._admit_sjf_locked()
            return
        i = 0
        while i < len(self._queue) and self._free_slots:
            p = self._queue[i]
            slot = self._fit_slot(p)
            if slot is not None:
                self._start_locked(i, slot)
                i = 0
                continue
            if p.bypassed >= self.max_bypass:
                break  # the oldest blocked request has waited long enough: no more back-filling
            i += 1

    def _admit_sjf_locked(self):
        while self._queue and self._free_slots:
            q = self._queue
            if q[0].bypassed >= self.max_bypass:
                order = [0]  # passed over often enough: the oldest goes next, or nothing does
            else:
                order = sorted(range(len(q)), key=lambda j: (q[j].req.count, j))
            for i in order:
                slot = self._fit_slot(q[i])
                if slot is not None:
                    self._start_locked(i, slot)
                    break
            else:
                return

    def _complete_locked(self):
        still = []
        for r in self._running:
            try:
                if not self.ex.done(r.handle):
                    still.append(r)
                    continue
                res = self.ex.finish(r.handle)
            except Exception as e:  # the request failed on completion: report it, release its slot and bytes
                self._bytes -= r.pend.footprint
                self._free_slots.append(r.slot)
                self.stats.failed += 1
                r.pend.fut.set_exception(e)
                continue
            t = self.clock()
            res.t_submit, res.t_admit, res.t_done, res.slot, res.tag = r.pend.t_submit, r.t_admit, t, r.slot, \
                r.pend.req.tag
            self._bytes -= r.pend.footprint
            self._free_slots.append(r.slot)
            self.stats.completed += 1
            self.stats.fragments += r.pend.req.count
            self.stats.latencies.append(res.latency)
            self.stats.waits.append(r.t_admit - r.pend.t_submit)
            self.stats.last_done = max(self.stats.last_done, t)
            r.pend.fut.set_result(res)
        self._running = still

    def _wait_loop(self, q):
        while True:
            handle = q.get()
            if handle is None:
                return
            try:
                self.ex.wait(handle)
            except Exception:  # finish() reports the failure on the scheduler thread
                pass
            with self._cv:
                self._cv.notify_all()

    def _wake_in(self) -> float:
        """How long the scheduler may sleep when a waiting thread, a submission or close will wake it: until the
        nearest admission deadline of a queued request, and briefly while requests are queued (to count client
        cancellations)."""
        t = 0.005 if self._queue else 0.05
        now = self.clock()
        for p in self._queue:
            if p.req.timeout is not None:
                t = min(t, max(0.0, p.t_submit + p.req.timeout - now) + 1e-4)
        return t

    def _loop(self):
        try:
            while True:
                with self._cv:
                    if self._stop and not self._queue and not self._running:
                        return
                    self._complete_locked()
                    self._admit_locked()
                    idle = not self._running and not self._queue
                    if self._blocking:
                        if not (idle and self._stop):
                            self._cv.wait(timeout=self._wake_in())
                        continue
                    if idle and not self._stop:
                        self._cv.wait(timeout=0.05)
                        continue
                time.sleep(self.poll_interval)
        finally:
            for q in self._wq:
                q.put(None)


def _slot_bytes(spec, count):
    """(workspace, coefficient) bytes a slot needs for a frame of this description and fragment count."""
    from . import wt as _wt
    n_el = 1
    for d in spec.coeff_shape():
        n_el *= d
    return _wt.workspace_bytes(spec, max(count, 1)), n_el * _wt.TORCH_DTYPES[spec.dtype].itemsize


class _WsView:
    """A workspace borrowed from a larger per-slot buffer (the ABI derives the layout from the byte count)."""

    def __init__(self, buf, nbytes):
        import ctypes as C
        self.buf = buf
        self.nbytes = int(nbytes)
        self.ptr = C.c_void_p(buf.data_ptr())


class GpuExecutor:
    """Runs requests on the GPU: one HIP stream per slot (default priority); per slot one resident workspace and
    one resident coefficient buffer, grown to the largest request it has taken (and released by ``trim`` when the
    scheduler needs the memory), shared by every frame description; completion observed through an event recorded
    after the request's work.

    Streams: ``prepare`` runs on the submitting thread, allocates the request's result buffers from that thread's
    current stream and records an event there; the slot stream waits for that event before reading the fragments,
    so inputs still being produced on the client's stream are complete. The fragment and result tensors are
    marked as used by the slot stream (``record_stream``), so the caching allocator does not hand their memory to
    other work before the slot's kernels are done with it, whichever stream frees them.

    Completion is polled (``done``); the executor has no ``wait``. Threads blocked in ``hipEventSynchronize`` on
    the slots' completion events (through torch or through ctypes with the interpreter lock released) held up the
    client's submissions, whose event records waited behind them: at 0.8 of the solo capacity submissions fell
    up to 85 ms behind the arrival trace and the median latency from arrival rose from 7 to 23 ms."""

    def __init__(self, slots: int = 3, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.ws = [None] * slots
        self.cf = [None] * slots

    def _spec(self, req):
        from . import wt as _wt
        return _wt.FrameSpec(req.width, req.height, req.rank, req.channels, req.dtype)

    def footprint(self, req: FrameRequest) -> int:
        """Bytes the request holds besides the slot's resident buffers: its fragment stream, its composite and,
        when asked for, its coefficient copy."""
        spec = self._spec(req)
        fr = req.count * (4 + 4 + 4 * req.channels + 12)
        return fr + spec.pixels * 12 + (_slot_bytes(spec, req.count)[1] if req.want_coeffs else 0)

    def growth(self, slot, req: FrameRequest) -> int:
        """Bytes slot's resident buffers must grow by to take req (the full need for slot None or an empty slot)."""
        need_ws, need_cf = _slot_bytes(self._spec(req), req.count)
        have_ws = 0 if slot is None or self.ws[slot] is None else self.ws[slot].numel()
        have_cf = 0 if slot is None or self.cf[slot] is None else self.cf[slot].numel()
        return max(0, need_ws - have_ws) + max(0, need_cf - have_cf)

    def resident_bytes(self) -> int:
        return sum(b.numel() for b in self.ws + self.cf if b is not None)

    def reserve(self, width: int, height: int, rank: int, count: int, channels: int = 1, dtype: str = "f32"):
        """Grow every slot's resident buffers to hold a request of this description and fragment count now, so that
        requests up to that size allocate nothing when they are launched (the buffers count against the server's
        budget as resident bytes)."""
        from . import wt as _wt
        need_ws, need_cf = _slot_bytes(_wt.FrameSpec(width, height, rank, channels, dtype), count)
        torch = self.torch
        for k, s in enumerate(self.streams):
            with torch.cuda.stream(s):
                if self.ws[k] is None or self.ws[k].numel() < need_ws:
                    self.ws[k] = None
                    self.ws[k] = torch.empty(need_ws, dtype=torch.uint8, device=self.device)
                if self.cf[k] is None or self.cf[k].numel() < need_cf:
                    self.cf[k] = None
                    self.cf[k] = torch.empty(need_cf, dtype=torch.uint8, device=self.device)

    def trim(self, slot: int):
        """Release an idle slot's buffers (its stream's earlier work is ordered before any reuse of the memory)."""
        self.ws[slot] = None
        self.cf[slot] = None

    def prepare(self, req: FrameRequest):
        torch = self.torch
        spec = self._spec(req)
        from . import wt as _wt
        client = torch.cuda.current_stream(self.device)
        out = req.out
        if out is None:
            out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=self.device)
        elif (not isinstance(out, torch.Tensor) or out.dtype != torch.float32 or out.device != self.device or
              tuple(out.shape) != (spec.pixels, 3) or not out.is_contiguous()):
            raise ValueError("FrameRequest.out must be a contiguous [%d, 3] float32 tensor on %s" %
                             (spec.pixels, self.device))
        kept = torch.empty(spec.coeff_shape(), dtype=_wt.TORCH_DTYPES[spec.dtype], device=self.device) \
            if req.want_coeffs else None
        ready = torch.cuda.Event()
        ready.record(client)
        return (out, kept, ready)

    def _buffers(self, slot, req, spec):
        from . import wt as _wt
        torch = self.torch
        need_ws, need_cf = _slot_bytes(spec, req.count)
        with torch.cuda.stream(self.streams[slot]):
            if self.ws[slot] is None or self.ws[slot].numel() < need_ws:
                self.ws[slot] = None
                self.ws[slot] = torch.empty(need_ws, dtype=torch.uint8, device=self.device)
            if self.cf[slot] is None or self.cf[slot].numel() < need_cf:
                self.cf[slot] = None
                self.cf[slot] = torch.empty(need_cf, dtype=torch.uint8, device=self.device)
        ws = _WsView(self.ws[slot], self.ws[slot].numel())
        coeffs = self.cf[slot][:need_cf].view(_wt.TORCH_DTYPES[spec.dtype]).view(spec.coeff_shape())
        return ws, coeffs

    def launch(self, req: FrameRequest, slot: int, token=None):
        from . import wt as _wt
        torch = self.torch
        if token is None:
            token = self.prepare(req)
        out, kept, ready = token
        spec = self._spec(req)
        s = self.streams[slot]
        s.wait_event(ready)  # the inputs as the client's stream left them at submit
        for t in (req.frags.pixel, req.frags.depth, req.frags.alpha, req.frags.rgb, out, kept):
            if t is not None:
                t.record_stream(s)
        ws, coeffs = self._buffers(slot, req, spec)
        with torch.cuda.stream(s):
            _wt.render(spec, req.frags, req.bg, ws, out=out, coeffs=coeffs, stream=s)
            if kept is not None:
                kept.copy_(coeffs)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, out, kept)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> FrameResult:
        ev, out, kept = handle
        return FrameResult(out=out, coeffs=kept)
