"""Continuous-batching server for wavelet resolves.

Frames of different sizes, ranks and coefficient storage types arrive as requests. The scheduler admits a request
as soon as an execution slot is free and its HBM footprint fits the remaining budget, launches it on that slot's
HIP stream, and keeps polling the device: requests that arrive while others run are admitted as slots and memory
free up, and their work overlaps on the GPU. Per-slot buffers (workspace and coefficient array) stay resident and
are reused across requests of the same frame description. Latency is measured from arrival (submit) to the moment
the completion event is observed.

The scheduler is independent of the device: it drives an executor with ``footprint``, ``launch``, ``done`` and
``finish``. :class:`GpuExecutor` runs the library; tests drive the scheduler with a CPU executor.
"""
from __future__ import annotations

import collections
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


@dataclass
class _Pending:
    req: FrameRequest
    fut: Future
    t_submit: float
    footprint: int
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
                "fragments": self.fragments,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "fragments_per_s": self.fragments / span,
                "queued": int((wait > 1.0).sum()), "wait_p50_ms": float(np.percentile(wait, 50)),
                "wait_p99_ms": float(np.percentile(wait, 99)),
                "max_inflight": self.max_inflight, "max_bytes_inflight": self.max_bytes_inflight}


class Server:
    """Admission by HBM footprint and free slots; FIFO with bounded back-filling (a request that does not fit
    may be passed by later, smaller ones at most ``max_bypass`` times, after which admission waits for it)."""

    def __init__(self, executor, slots: int = 3, budget_bytes: int = 96 << 30, max_bypass: int = 8,
                 poll_interval: float = 0.0002, clock=time.perf_counter):
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
        self._cv = threading.Condition()
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="wt-serve", daemon=True)
        self._thread.start()

    # -- client side --------------------------------------------------------------------------------------
    def submit(self, req: FrameRequest) -> Future:
        fut: Future = Future()
        t = self.clock()
        fp = int(self.ex.footprint(req))
        with self._cv:
            if self._stop:
                raise RuntimeError("the server is closed")
            self.stats.first_submit = min(self.stats.first_submit, t)
            if fp > self.budget:
                self.stats.rejected += 1
                fut.set_exception(RequestTooLarge("request needs %d bytes, the budget is %d" % (fp, self.budget)))
                return fut
            self._queue.append(_Pending(req, fut, t, fp))
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
    def _admit_locked(self):
        i = 0
        while i < len(self._queue) and self._free_slots:
            p = self._queue[i]
            if self._bytes + p.footprint <= self.budget:
                del self._queue[i]
                slot = self._free_slots.pop()
                self._bytes += p.footprint
                t = self.clock()
                try:
                    handle = self.ex.launch(p.req, slot)
                except Exception as e:  # launch failure: report to the client, release resources
                    self._bytes -= p.footprint
                    self._free_slots.append(slot)
                    self.stats.failed += 1
                    p.fut.set_exception(e)
                    continue
                self._running.append(_Running(p, slot, handle, t))
                self.stats.max_inflight = max(self.stats.max_inflight, len(self._running))
                self.stats.max_bytes_inflight = max(self.stats.max_bytes_inflight, self._bytes)
                # requests ahead of this one were passed over once more
                for q in list(self._queue)[:i]:
                    q.bypassed += 1
                i = 0
                continue
            if p.bypassed >= self.max_bypass:
                break  # the oldest blocked request has waited long enough: no more back-filling
            i += 1

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

    def _loop(self):
        while True:
            with self._cv:
                if self._stop and not self._queue and not self._running:
                    return
                self._complete_locked()
                self._admit_locked()
                idle = not self._running and not self._queue
                if idle and not self._stop:
                    self._cv.wait(timeout=0.05)
                    continue
            time.sleep(self.poll_interval)


def request_footprint(width, height, rank, channels, dtype, count, stream_bytes=True):
    """HBM bytes a request holds while it runs: its fragment stream (if counted), the binning workspace, the
    coefficient array and the composite."""
    from . import wt as _wt
    spec = _wt.FrameSpec(width, height, rank, channels, dtype)
    sbytes = {"f32": 4, "f16": 2, "bf16": 2, "e5b9g9r9": 4}[dtype]
    ws = _wt.workspace_bytes(spec, max(count, 1))
    fr = count * (4 + 4 + 4 * channels + 12) if stream_bytes else 0
    coeff_elems = 1
    for d in spec.coeff_shape():
        coeff_elems *= d
    return fr + ws + coeff_elems * sbytes + spec.pixels * 12


class _WsView:
    """A workspace borrowed from a larger per-slot buffer (the ABI derives the layout from the byte count)."""

    def __init__(self, buf, nbytes):
        import ctypes as C
        self.buf = buf
        self.nbytes = int(nbytes)
        self.ptr = C.c_void_p(buf.data_ptr())


class GpuExecutor:
    """Runs requests on the GPU: one HIP stream per slot (default priority); per slot one resident workspace and
    one resident coefficient buffer, grown to the largest request seen and shared by every frame description;
    completion observed through an event recorded after the request's work."""

    def __init__(self, slots: int = 3, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.ws = [None] * slots
        self.cf = [None] * slots

    def footprint(self, req: FrameRequest) -> int:
        return request_footprint(req.width, req.height, req.rank, req.channels, req.dtype, req.count)

    def _buffers(self, slot, req, spec):
        from . import wt as _wt
        torch = self.torch
        need_ws = _wt.workspace_bytes(spec, max(req.count, 1))
        n_el = 1
        for d in spec.coeff_shape():
            n_el *= d
        need_cf = n_el * _wt.TORCH_DTYPES[spec.dtype].itemsize
        with torch.cuda.stream(self.streams[slot]):
            if self.ws[slot] is None or self.ws[slot].numel() < need_ws:
                self.ws[slot] = torch.empty(need_ws, dtype=torch.uint8, device=self.device)
            if self.cf[slot] is None or self.cf[slot].numel() < need_cf:
                self.cf[slot] = torch.empty(need_cf, dtype=torch.uint8, device=self.device)
        ws = _WsView(self.ws[slot], self.ws[slot].numel())
        coeffs = self.cf[slot][:need_cf].view(_wt.TORCH_DTYPES[spec.dtype]).view(spec.coeff_shape())
        return ws, coeffs

    def launch(self, req: FrameRequest, slot: int):
        from . import wt as _wt
        torch = self.torch
        spec = _wt.FrameSpec(req.width, req.height, req.rank, req.channels, req.dtype)
        s = self.streams[slot]
        s.wait_stream(torch.cuda.current_stream(self.device))  # inputs produced on the client's stream
        ws, coeffs = self._buffers(slot, req, spec)
        with torch.cuda.stream(s):
            out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=self.device)
            _wt.render(spec, req.frags, req.bg, ws, out=out, coeffs=coeffs, stream=s)
            kept = coeffs.clone() if req.want_coeffs else None
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, out, kept)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> FrameResult:
        ev, out, kept = handle
        return FrameResult(out=out, coeffs=kept)
