"""Serving loop: continuous batching of arriving depth maps.

Requests arrive one frame at a time (device-resident input tensors).  The
server

* admits a request when its output buffer fits in the device-memory budget
  (output bytes of admitted requests whose outputs have not been released);
  requests wait in arrival order otherwise, and are rejected only when the
  waiting queue is full or a frame alone exceeds the budget.  Output buffers
  are resident: released ones are reused, so the steady state allocates
  nothing;
* groups admitted requests into size buckets (frame shape rounded up to
  64 x 64, plus the parameter set), because one launch costs as much as its
  largest frames;
* launches a batch whenever one of its execution slots (a stream each) is
  free: the bucket of the oldest admitted request, up to `max_batch` of its
  requests in arrival order.  New arrivals are admitted and launched on
  another slot while earlier batches still run, so their work overlaps on the
  device (continuous batching, not a queue in front of one batch);
* polls the end-of-batch events; a request's latency is the time its event
  was observed complete minus its scheduled arrival;
* handles failures: a launch (or an event query) that raises marks its
  batch failed, and each of its requests is retried once alone; a request
  that fails alone is marked failed with the error, and its memory leaves
  the budget.  Requests can be cancelled, and requests still waiting for a
  launch when their timeout passes are dropped with status "timeout".

Memory admission counts, besides the outputs of admitted requests, what the
executor keeps resident (workspaces of its engines, released output buffers
kept for reuse); when nothing runs and the next request does not fit, the
executor is asked to drop idle resident memory first.

Stream order: a request's frame may come from work on another stream.  The
GPU executors note the submitting thread's current stream when a request is
submitted (or take the client's own event); before a launch reads the
frames, the slot stream waits for an event recorded on each such stream (one
per distinct stream of the batch), which covers all work the client queued
there before submitting.  An output buffer the client releases is reused
only after an event recorded on the releasing thread's current stream; one
the server releases itself (outputs not kept) needs none, as the batch that
wrote it has completed and nothing else read it.

Every frame is completed independently of the others in its batch (Sec. II),
so a result does not depend on what it was batched with.

Executors do the device work: `GraphExecutor` (one GraphBatch per slot and
bucket, replayed as a HIP graph) and `PerFrameExecutor` (the plain path: one
ipb_complete_ws per request on a single stream, in arrival order).  Tests
drive the scheduler with a host-only executor.
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import math
import time
from typing import Callable, Deque, Dict, Hashable, List, Optional, Sequence, Tuple

import numpy as np

try:
    import torch
except ImportError:  # the scheduler itself needs no torch
    torch = None

BUCKET = 64


def default_bucket(shape: Tuple[int, int]) -> Tuple[int, int]:
    H, W = shape
    return (-(-H // BUCKET) * BUCKET, -(-W // BUCKET) * BUCKET)


@dataclasses.dataclass(eq=False)
class Request:
    rid: int
    frame: object                      # device tensor, H x W float32
    shape: Tuple[int, int]
    arrival: float                     # scheduled arrival, seconds on the server clock
    params: object = None
    bucket: Hashable = None
    nbytes: int = 0
    # queued, admitted, running, done, released, rejected, failed, cancelled, timeout
    status: str = "queued"
    out: object = None
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    deadline: float = math.inf         # launch by then, or the request times out
    ready: object = None               # event after the work that produced `frame` (GPU executors)
    src: object = None                 # stream current when submitted (GPU executors)
    attempts: int = 0                  # launches that failed
    solo: bool = False                 # to be launched alone (a retry after a failed batch)
    cancelled: bool = False            # cancelled while running: released when it completes
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Executor:
    """Device side of the server: `slots` independent execution slots.
    `in_order`: batches finish in launch order (a single stream), so the
    server polls only the oldest one."""
    slots: int = 1
    in_order: bool = False

    def submitted(self, req: Request) -> None:
        """A request entered the server (GPU executors note the stream order
        of its frame here)."""

    def launch(self, slot: int, bucket: Hashable, reqs: Sequence[Request]) -> object:
        raise NotImplementedError

    def ready(self, handle: object) -> bool:
        raise NotImplementedError

    def outputs(self, handle: object) -> List[object]:
        raise NotImplementedError

    def recycle(self, outs: Sequence[object], by_client: bool = True) -> None:
        """Output buffers handed back: by the client (who may still have
        reads of them queued on its current stream), or by the server itself
        right after their batch completed."""

    def resident_bytes(self) -> int:
        """Device memory the executor keeps between batches."""
        return 0

    def trim(self, target: int) -> None:
        """Drop idle resident memory until at most `target` bytes remain (if
        it can); called only while no batch runs."""


class Server:
    def __init__(self, executor: Executor, mem_budget: int, max_batch: int = 16, max_queue: int = 100000,
                 bucket_fn: Callable[[Tuple[int, int]], Hashable] = default_bucket,
                 clock: Callable[[], float] = time.perf_counter, keep_outputs: bool = True,
                 timeout: Optional[float] = None):
        if mem_budget <= 0 or max_batch < 1:
            raise ValueError("mem_budget and max_batch must be positive")
        if timeout is not None and not timeout > 0:
            raise ValueError("timeout must be positive")
        self.ex = executor
        self.mem_budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.max_queue = int(max_queue)
        self.bucket_fn = bucket_fn
        self.clock = clock
        self.keep_outputs = keep_outputs
        self.timeout = timeout
        self.t0 = clock()
        self.waiting: Deque[Request] = collections.deque()          # not yet admitted, arrival order
        self.admitted: Dict[Hashable, Deque[Request]] = collections.OrderedDict()
        self.retry: Deque[Request] = collections.deque()            # admitted, to be launched alone
        self.in_use = 0                                             # admitted, unreleased output bytes
        self.running: "collections.OrderedDict[int, Tuple[object, List[Request]]]" = collections.OrderedDict()
        self.free_slots: List[int] = list(range(executor.slots - 1, -1, -1))
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.failed: List[Request] = []
        self.cancelled: List[Request] = []
        self.timed_out: List[Request] = []
        self.batches = 0
        self.failed_batches = 0
        self.launch_s = 0.0                                         # host seconds spent in launches
        self.peak_in_use = 0
        self._next_id = 0
        self._deadlines = False                                     # some request has a finite deadline

    def now(self) -> float:
        return self.clock() - self.t0

    # ---------------------------------------------------------------- intake --
    def submit(self, frame, arrival: Optional[float] = None, params=None,
               shape: Optional[Tuple[int, int]] = None, ready=None, timeout: Optional[float] = None) -> Request:
        """Queue one frame.  ready: an event marking the end of the work that
        produced the frame (GPU executors otherwise record one on the current
        stream); timeout: seconds from arrival by which the request must be
        launched (default: the server's)."""
        shape = tuple(shape if shape is not None else frame.shape)
        req = Request(self._next_id, frame, shape, self.now() if arrival is None else arrival, params)
        self._next_id += 1
        req.bucket = (self.bucket_fn(shape), _params_key(params))
        req.nbytes = 4 * shape[0] * shape[1]
        t_out = timeout if timeout is not None else self.timeout
        if t_out is not None:
            req.deadline = req.arrival + t_out
            self._deadlines = True
        if req.nbytes > self.mem_budget or len(self.waiting) >= self.max_queue:
            req.status = "rejected"
            self.rejected.append(req)
            return req
        req.ready = ready
        self.ex.submitted(req)
        self.waiting.append(req)
        return req

    def cancel(self, req: Request) -> bool:
        """Cancel a request.  One that waits or is admitted leaves at once
        (status "cancelled", its memory leaves the budget); one that runs
        cannot be stopped on the device: it is marked, and when its batch
        completes its output is released and its status is "cancelled".
        Returns False if the request had already finished."""
        if req.status == "queued":
            self.waiting.remove(req)
        elif req.status == "admitted":
            if req.solo:
                self.retry.remove(req)
            else:
                self.admitted[req.bucket].remove(req)
            self.in_use -= req.nbytes
        elif req.status == "running":
            req.cancelled = True
            return True
        else:
            return False
        req.status = "cancelled"
        self.cancelled.append(req)
        return True

    # ------------------------------------------------------------ scheduling --
    def _finish(self, reqs: Sequence[Request], outs: Sequence[object], t: float) -> List[Request]:
        done, back = [], []
        for r, o in zip(reqs, outs):
            r.t_done = t
            r.out = o
            r.status = "done"
            if r.cancelled:
                back.append(r)
                self.cancelled.append(r)
                continue
            done.append(r)
            if not self.keep_outputs:
                back.append(r)
        self.release_many(back, by_client=False)
        for r in back:
            if r.cancelled:
                r.status = "cancelled"
        self.done.extend(done)
        return done

    def _fail(self, reqs: Sequence[Request], exc: BaseException) -> None:
        """A batch failed (its launch or its completion raised): requests
        that failed in a batch are retried once alone; one that failed alone
        is marked failed (cancelled ones just leave)."""
        self.failed_batches += 1
        for r in reqs:
            r.attempts += 1
            if r.cancelled:
                r.status = "cancelled"
                self.in_use -= r.nbytes
                self.cancelled.append(r)
            elif r.solo or r.attempts >= 2:
                r.status = "failed"
                r.error = f"{type(exc).__name__}: {exc}"
                self.in_use -= r.nbytes
                self.failed.append(r)
            else:
                r.status = "admitted"
                r.solo = True
                self.retry.append(r)

    def _poll(self) -> List[Request]:
        finished = []
        for s, (handle, reqs) in list(self.running.items()):
            try:
                ok = self.ex.ready(handle)
                outs = self.ex.outputs(handle) if ok else None
            except Exception as exc:          # the batch's device work failed
                del self.running[s]
                self.free_slots.append(s)
                self._fail(reqs, exc)
                continue
            if not ok:
                if self.ex.in_order:
                    break
                continue
            del self.running[s]
            self.free_slots.append(s)
            finished.extend(self._finish(reqs, outs, self.now()))
        return finished

    def _expire(self) -> None:
        """Requests not launched by their deadline time out."""
        if not self._deadlines:
            return
        t = self.now()
        keep = collections.deque()
        for r in self.waiting:
            if r.deadline < t:
                r.status = "timeout"
                self.timed_out.append(r)
            else:
                keep.append(r)
        self.waiting = keep
        for q in list(self.admitted.values()) + [self.retry]:
            late = [r for r in q if r.deadline < t]
            for r in late:
                q.remove(r)
                r.status = "timeout"
                self.in_use -= r.nbytes
                self.timed_out.append(r)

    def _reserved(self) -> int:
        return self.in_use + self.ex.resident_bytes()

    def _admit(self) -> None:
        while self.waiting:
            need = self.waiting[0].nbytes
            if self._reserved() + need > self.mem_budget:
                if self.running or any(self.admitted.values()) or self.retry:
                    break
                # nothing runs: let the executor drop idle resident memory
                self.ex.trim(max(0, self.mem_budget - self.in_use - need))
                if self._reserved() + need > self.mem_budget:
                    break
            r = self.waiting.popleft()
            r.status = "admitted"
            r.t_admit = self.now()
            self.in_use += r.nbytes
            self.admitted.setdefault(r.bucket, collections.deque()).append(r)
        self.peak_in_use = max(self.peak_in_use, self.in_use)

    def _launch(self) -> None:
        while self.free_slots:
            if self.retry:
                reqs = [self.retry.popleft()]           # a retry runs alone
                bucket = reqs[0].bucket
            else:
                live = [(q[0].rid, b) for b, q in self.admitted.items() if q]
                if not live:
                    return
                _, bucket = min(live, key=lambda v: v[0])      # the bucket of the oldest admitted request
                q = self.admitted[bucket]
                reqs = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
            s = self.free_slots.pop()
            t = self.now()
            for r in reqs:
                r.status = "running"
                r.t_launch = t
            try:
                handle = self.ex.launch(s, bucket, reqs)
            except Exception as exc:                   # nothing of the batch was queued, or its queue failed
                self.free_slots.append(s)
                self._fail(reqs, exc)
                continue
            finally:
                self.launch_s += self.now() - t
            self.running[s] = (handle, reqs)
            self.batches += 1

    def step(self) -> List[Request]:
        """One scheduling round: collect finished batches, drop requests past
        their deadline, admit, launch."""
        finished = self._poll()
        self._expire()
        self._admit()
        self._launch()
        return finished

    def idle(self) -> bool:
        return not self.waiting and not any(self.admitted.values()) and not self.running and not self.retry

    def stalled(self) -> bool:
        """Requests wait, nothing runs or is admitted, and the next one does
        not fit even after the executor dropped its idle memory: only
        releasing outputs can make progress."""
        return (bool(self.waiting) and not self.running and not any(self.admitted.values()) and not self.retry
                and self._reserved() + self.waiting[0].nbytes > self.mem_budget)

    def drain(self, timeout: float = 60.0) -> None:
        t_end = self.now() + timeout
        while not self.idle():
            self.step()
            if self.stalled():
                raise RuntimeError("memory budget held by unreleased outputs")
            if self.now() > t_end:
                raise TimeoutError("server did not drain")

    def release(self, req: Request) -> None:
        """Hand a finished request's output buffer back (its bytes leave the
        budget; the buffer is reused once the work queued so far on the
        current stream, such as the client's reads of it, is done)."""
        self.release_many([req])

    def release_many(self, reqs: Sequence[Request], by_client: bool = True) -> None:
        outs = []
        for req in reqs:
            if req.status != "done" or req.out is None:
                continue
            outs.append(req.out)
            req.out = None
            req.status = "released"
            self.in_use -= req.nbytes
        if outs:
            self.ex.recycle(outs, by_client)

    # ------------------------------------------------------------- statistics --
    def stats(self, since: float = 0.0) -> dict:
        """Latency percentiles (arrival to observed completion), the wait
        before launch and the launch-to-completion service time, over the
        requests that arrived at or after `since`."""
        span = [r for r in self.done if r.arrival >= since]
        lat = np.array([r.latency for r in span], np.float64)
        out = {"completed": int(lat.size), "rejected": len(self.rejected), "failed": len(self.failed),
               "cancelled": len(self.cancelled), "timed_out": len(self.timed_out), "batches": self.batches,
               "failed_batches": self.failed_batches, "peak_mem_bytes": int(self.peak_in_use)}
        if lat.size:
            wait = np.array([r.t_launch - r.arrival for r in span], np.float64)
            svc = np.array([r.t_done - r.t_launch for r in span], np.float64)
            t_first = min(r.arrival for r in span)
            t_last = max(r.t_done for r in span)
            out.update(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                       mean_ms=float(lat.mean() * 1e3), max_ms=float(lat.max() * 1e3),
                       wait_p99_ms=float(np.percentile(wait, 99) * 1e3),
                       service_p50_ms=float(np.percentile(svc, 50) * 1e3),
                       service_p99_ms=float(np.percentile(svc, 99) * 1e3),
                       frames_per_batch=float(len(self.done) / max(self.batches, 1)),
                       host_launch_us=float(1e6 * self.launch_s / max(self.batches, 1)),
                       throughput_fps=float(lat.size / max(t_last - t_first, 1e-9)))
        return out


def _params_key(params) -> Hashable:
    if params is None:
        return None
    if dataclasses.is_dataclass(params):
        return tuple(dataclasses.astuple(params))
    return params


def run_trace(server: Server, frames: Sequence, arrivals: Sequence[float], params: Sequence = None,
              warmup: float = 0.0) -> dict:
    """Feed frames at their arrival times (seconds from now) in real time,
    run the scheduler until every request finished, and return statistics
    over the requests that arrived after `warmup` seconds."""
    n = len(frames)
    gc_was = gc.isenabled()
    gc.disable()                      # no collector pauses inside the timed loop
    try:
        base = server.now()
        i = 0
        while i < n or not server.idle():
            t = server.now() - base
            while i < n and arrivals[i] <= t:
                server.submit(frames[i], arrival=base + float(arrivals[i]), params=params[i] if params else None)
                i += 1
            server.step()
            if i >= n and server.stalled():
                raise RuntimeError("memory budget held by unreleased outputs")
    finally:
        if gc_was:
            gc.enable()
    return server.stats(since=base + warmup)


# ------------------------------------------------------------- executors --

class BufferPool:
    """Resident output buffers by shape: a released buffer is reused by the
    next request of that shape, so steady-state serving allocates nothing.
    A buffer comes back only after the batch that wrote it completed and the
    client released it; the release records an event on the releasing
    thread's current stream (where the client read the buffer), and the next
    writer's stream waits for it.  New buffers are allocated under the stream
    that first writes them."""

    def __init__(self, device):
        self.device = device
        self.free: Dict[Tuple[int, int], List[Tuple[object, object]]] = collections.defaultdict(list)
        self.allocated = 0
        self.free_bytes = 0

    def get(self, shape: Tuple[int, int], stream):
        """A buffer of `shape` that `stream` may write (the stream is made to
        wait for the buffer's last reader)."""
        lst = self.free.get(shape)
        if lst:
            buf, ev = lst.pop()
            self.free_bytes -= 4 * shape[0] * shape[1]
            if ev is not None:
                stream.wait_event(ev)
            return buf
        self.allocated += 1
        with torch.cuda.stream(stream):
            return torch.empty(shape, dtype=torch.float32, device=self.device)

    def put(self, bufs: Sequence[object], by_client: bool = True) -> None:
        """Buffers back to the pool.  by_client: the releasing thread may
        still have reads of them queued on its current stream, so their next
        writer waits for an event recorded there; otherwise (the server
        releases outputs no client saw) their last use has completed."""
        if not bufs:
            return
        ev = None
        if by_client:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(self.device))
        for b in bufs:
            self.free[tuple(b.shape)].append((b, ev))
            self.free_bytes += 4 * b.numel()

    def clear(self) -> None:
        self.free.clear()
        self.free_bytes = 0


class _InputOrder:
    """Orders a launch stream after the work that produced its frames: the
    client's events, and, for requests without one, an event recorded now on
    each stream that was current at their submission (once per distinct
    stream; an event recorded later than the submission covers the client's
    work queued before it).  One event object is reused: a stream's wait
    takes the event's state at the time of the call."""

    def __init__(self):
        self.ev = torch.cuda.Event()

    def wait(self, stream, reqs: Sequence[Request]) -> None:
        seen = set()
        for r in reqs:
            if r.ready is not None:
                if id(r.ready) not in seen:
                    seen.add(id(r.ready))
                    stream.wait_event(r.ready)
            elif r.src is not None:
                h = r.src.cuda_stream
                if h not in seen and h != stream.cuda_stream:
                    seen.add(h)
                    self.ev.record(r.src)
                    stream.wait_event(self.ev)


def _note_submit(req: Request, device, order_inputs: bool) -> None:
    """Note the submitting thread's current stream (the client's event, if it
    gave one, takes precedence).  order_inputs False: the client guarantees
    its frames are complete when submitted (e.g. resident frames made before
    a synchronisation), so nothing is noted."""
    if req.ready is None and order_inputs:
        req.src = torch.cuda.current_stream(device)


class GraphExecutor(Executor):
    """Batches replayed as HIP graphs, each slot on its own stream of
    default priority.  Per slot and bucket there is one GraphBatch per
    capacity tier (e.g. 1, 4 and 16 frames): a batch runs on the smallest
    tier that holds it, so a lone request under light load does not pay for
    the launch grid of a full batch.  With `direct_single`, a lone request
    skips the graph (and its plan copy) and goes straight to ipb_complete_ws
    on the slot's stream, with a workspace resident per slot.  order_inputs:
    launches wait for the streams the frames were submitted on (see the
    module notes); False for clients whose frames are complete when
    submitted."""

    def __init__(self, slots: int = 2, max_batch: int = 16, device=None, default_params=None,
                 tiers: Optional[Sequence[int]] = None, direct_single: bool = True, order_inputs: bool = True):
        from .api import Params
        self.direct_single = direct_single
        self.order_inputs = order_inputs
        self.ws: Dict[int, object] = {}
        self.ws_bytes: Dict[int, int] = {}
        self.cparams: Dict[Hashable, object] = {}
        self.slots = slots
        self.max_batch = max_batch
        if tiers is None:
            tiers = sorted({1, min(4, max_batch), max_batch})
        self.tiers = sorted(t for t in tiers if 1 <= t <= max_batch)
        if not self.tiers or self.tiers[-1] != max_batch:
            self.tiers.append(max_batch)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.default_params = default_params or Params()
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # engines by (slot, bucket, tier), least recently used first
        self.engines: "collections.OrderedDict[Tuple[int, Hashable, int], object]" = collections.OrderedDict()
        self.pool = BufferPool(self.device)
        self.order = _InputOrder()
        self._eng_bytes = 0        # workspaces and plans of the engines
        self._ws_total = 0         # the per-slot workspaces of lone requests

    def _engine(self, slot: int, bucket: Hashable, params, n: int):
        from .batch import GraphBatch
        tier = next(t for t in self.tiers if t >= n)
        key = (slot, bucket, tier)
        eng = self.engines.get(key)
        if eng is None:
            (Hb, Wb), _ = bucket
            eng = GraphBatch([(Hb, Wb)] * tier, params or self.default_params, device=self.device,
                             stream=self.streams[slot])
            self.engines[key] = eng
            self._eng_bytes += eng.ws_bytes + eng.plan_bytes
        else:
            self.engines.move_to_end(key)
        return eng

    def submitted(self, req: Request) -> None:
        _note_submit(req, self.device, self.order_inputs)

    def resident_bytes(self) -> int:
        """Engine workspaces and plans, the per-slot workspaces of lone
        requests and the released output buffers kept for reuse."""
        return self._eng_bytes + self._ws_total + self.pool.free_bytes

    def trim(self, target: int) -> None:
        """Drop pooled outputs, then least recently used engines and the
        per-slot workspaces, until at most `target` bytes stay resident (only
        called while nothing runs, so nothing dropped is in use)."""
        self.pool.clear()
        while self.engines and self.resident_bytes() > target:
            _, e = self.engines.popitem(last=False)
            self._eng_bytes -= e.ws_bytes + e.plan_bytes
        if self.resident_bytes() > target:
            self.ws.clear()
            self.ws_bytes.clear()
            self._ws_total = 0

    def warm(self, bucket_params: Sequence[Tuple[Hashable, object]]) -> None:
        """Capture the graphs of these buckets on every slot and tier ahead
        of time."""
        for bucket, params in bucket_params:
            (Hb, Wb), _ = bucket
            x = torch.zeros((Hb, Wb), dtype=torch.float32, device=self.device)
            torch.cuda.synchronize(self.device)
            for s in range(self.slots):
                for tier in self.tiers:
                    eng = self._engine(s, bucket, params, tier)
                    for _ in range(3):
                        eng.run([x]).synchronize()

    def _direct(self, slot: int, r: Request):
        import ctypes
        from . import _lib as L
        from .api import _workspace
        lib = L.lib()
        stream = self.streams[slot]
        key = _params_key(r.params)
        cp = self.cparams.get(key)
        if cp is None:
            cp = self.cparams[key] = (r.params or self.default_params).to_c()
        H, W = r.shape
        need = int(lib.ipb_workspace_bytes(H, W, ctypes.byref(cp)))
        if need > self.ws_bytes.get(slot, 0):
            with torch.cuda.stream(stream):
                self.ws[slot] = _workspace(need, self.device)
            self._ws_total += need - self.ws_bytes.get(slot, 0)
            self.ws_bytes[slot] = need
        o = self.pool.get(r.shape, stream)
        self.order.wait(stream, [r])
        L.check(lib.ipb_complete_ws(ctypes.c_void_p(r.frame.data_ptr()), H, W, ctypes.byref(cp),
                                    ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(self.ws[slot].data_ptr()),
                                    self.ws_bytes[slot], ctypes.c_void_p(stream.cuda_stream)), "ipb_complete_ws")
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev, [o]

    def launch(self, slot: int, bucket: Hashable, reqs: Sequence[Request]):
        if self.direct_single and len(reqs) == 1:
            return self._direct(slot, reqs[0])
        eng = self._engine(slot, bucket, reqs[0].params, len(reqs))
        outs = [self.pool.get(r.shape, eng.stream) for r in reqs]
        self.order.wait(eng.stream, reqs)
        ev = eng.run([r.frame for r in reqs], outs)
        return ev, outs

    def ready(self, handle) -> bool:
        return handle[0].query()

    def outputs(self, handle) -> List[object]:
        return handle[1]

    def recycle(self, outs: Sequence[object], by_client: bool = True) -> None:
        self.pool.put(outs, by_client)


class PerFrameExecutor(Executor):
    """The plain path: every request is one ipb_complete_ws call on a single
    stream as soon as it is admitted, so the device runs them in arrival
    order (one resident workspace serves them all).  `slots` bounds the
    requests in flight; order_inputs as for GraphExecutor."""

    in_order = True

    def __init__(self, slots: int = 4096, device=None, default_params=None, order_inputs: bool = True):
        from .api import Params
        self.slots = slots
        self.order_inputs = order_inputs
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.default_params = default_params or Params()
        self.stream = torch.cuda.Stream(device=self.device)
        self.ws = None
        self.ws_bytes = 0
        self.cparams: Dict[Hashable, object] = {}
        self.pool = BufferPool(self.device)
        self.order = _InputOrder()

    def launch(self, slot: int, bucket: Hashable, reqs: Sequence[Request]):
        import ctypes
        from . import _lib as L
        from .api import _workspace
        lib = L.lib()
        h = ctypes.c_void_p(self.stream.cuda_stream)
        outs = []
        for r in reqs:
            key = _params_key(r.params)
            cp = self.cparams.get(key)
            if cp is None:
                cp = self.cparams[key] = (r.params or self.default_params).to_c()
            H, W = r.shape
            need = int(lib.ipb_workspace_bytes(H, W, ctypes.byref(cp)))
            if need > self.ws_bytes:
                with torch.cuda.stream(self.stream):
                    self.ws = _workspace(need, self.device)
                self.ws_bytes = need
            o = self.pool.get(r.shape, self.stream)
            self.order.wait(self.stream, [r])
            L.check(lib.ipb_complete_ws(ctypes.c_void_p(r.frame.data_ptr()), H, W, ctypes.byref(cp),
                                        ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                        self.ws_bytes, h), "ipb_complete_ws")
            outs.append(o)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev, outs

    def submitted(self, req: Request) -> None:
        _note_submit(req, self.device, self.order_inputs)

    def resident_bytes(self) -> int:
        return self.ws_bytes + self.pool.free_bytes

    def trim(self, target: int) -> None:
        self.pool.clear()
        if self.resident_bytes() > target:
            self.ws, self.ws_bytes = None, 0

    def ready(self, handle) -> bool:
        return handle[0].query()

    def outputs(self, handle) -> List[object]:
        return handle[1]

    def recycle(self, outs: Sequence[object], by_client: bool = True) -> None:
        self.pool.put(outs, by_client)
