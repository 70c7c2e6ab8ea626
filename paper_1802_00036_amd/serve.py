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
  was observed complete minus its scheduled arrival.

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
    status: str = "queued"             # queued, admitted, running, done, rejected
    out: object = None
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Executor:
    """Device side of the server: `slots` independent execution slots.
    `in_order`: batches finish in launch order (a single stream), so the
    server polls only the oldest one."""
    slots: int = 1
    in_order: bool = False

    def launch(self, slot: int, bucket: Hashable, reqs: Sequence[Request]) -> object:
        raise NotImplementedError

    def ready(self, handle: object) -> bool:
        raise NotImplementedError

    def outputs(self, handle: object) -> List[object]:
        raise NotImplementedError

    def recycle(self, outs: Sequence[object]) -> None:
        """Output buffers the client has finished with."""


class Server:
    def __init__(self, executor: Executor, mem_budget: int, max_batch: int = 16, max_queue: int = 100000,
                 bucket_fn: Callable[[Tuple[int, int]], Hashable] = default_bucket,
                 clock: Callable[[], float] = time.perf_counter, keep_outputs: bool = True):
        if mem_budget <= 0 or max_batch < 1:
            raise ValueError("mem_budget and max_batch must be positive")
        self.ex = executor
        self.mem_budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.max_queue = int(max_queue)
        self.bucket_fn = bucket_fn
        self.clock = clock
        self.keep_outputs = keep_outputs
        self.t0 = clock()
        self.waiting: Deque[Request] = collections.deque()          # not yet admitted, arrival order
        self.admitted: Dict[Hashable, Deque[Request]] = collections.OrderedDict()
        self.in_use = 0                                             # admitted, unreleased output bytes
        self.running: "collections.OrderedDict[int, Tuple[object, List[Request]]]" = collections.OrderedDict()
        self.free_slots: List[int] = list(range(executor.slots - 1, -1, -1))
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.batches = 0
        self.launch_s = 0.0                                         # host seconds spent in launches
        self.peak_in_use = 0
        self._next_id = 0

    def now(self) -> float:
        return self.clock() - self.t0

    # ---------------------------------------------------------------- intake --
    def submit(self, frame, arrival: Optional[float] = None, params=None,
               shape: Optional[Tuple[int, int]] = None) -> Request:
        shape = tuple(shape if shape is not None else frame.shape)
        req = Request(self._next_id, frame, shape, self.now() if arrival is None else arrival, params)
        self._next_id += 1
        req.bucket = (self.bucket_fn(shape), _params_key(params))
        req.nbytes = 4 * shape[0] * shape[1]
        if req.nbytes > self.mem_budget or len(self.waiting) >= self.max_queue:
            req.status = "rejected"
            self.rejected.append(req)
            return req
        self.waiting.append(req)
        return req

    # ------------------------------------------------------------ scheduling --
    def _poll(self) -> List[Request]:
        finished = []
        for s, (handle, reqs) in list(self.running.items()):
            if not self.ex.ready(handle):
                if self.ex.in_order:
                    break
                continue
            t = self.now()
            outs = self.ex.outputs(handle)
            for r, o in zip(reqs, outs):
                r.t_done = t
                r.status = "done"
                r.out = o
                if not self.keep_outputs:
                    self.release(r)
            del self.running[s]
            self.free_slots.append(s)
            self.done.extend(reqs)
            finished.extend(reqs)
        return finished

    def _admit(self) -> None:
        while self.waiting and self.in_use + self.waiting[0].nbytes <= self.mem_budget:
            r = self.waiting.popleft()
            r.status = "admitted"
            r.t_admit = self.now()
            self.in_use += r.nbytes
            self.admitted.setdefault(r.bucket, collections.deque()).append(r)
        self.peak_in_use = max(self.peak_in_use, self.in_use)

    def _launch(self) -> None:
        while self.free_slots:
            live = [(q[0].rid, b) for b, q in self.admitted.items() if q]
            if not live:
                return
            s = self.free_slots.pop()
            _, bucket = min(live, key=lambda v: v[0])      # the bucket of the oldest admitted request
            q = self.admitted[bucket]
            reqs = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
            t = self.now()
            for r in reqs:
                r.status = "running"
                r.t_launch = t
            handle = self.ex.launch(s, bucket, reqs)
            self.launch_s += self.now() - t
            self.running[s] = (handle, reqs)
            self.batches += 1

    def step(self) -> List[Request]:
        """One scheduling round: collect finished batches, admit, launch."""
        finished = self._poll()
        self._admit()
        self._launch()
        return finished

    def idle(self) -> bool:
        return not self.waiting and not any(self.admitted.values()) and not self.running

    def stalled(self) -> bool:
        """Requests wait, nothing runs or is admitted, and the next one does
        not fit: only releasing outputs can make progress."""
        return (bool(self.waiting) and not self.running and not any(self.admitted.values())
                and self.in_use + self.waiting[0].nbytes > self.mem_budget)

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
        budget; the buffer is reused)."""
        if req.status != "done" or req.out is None:
            return
        self.ex.recycle([req.out])
        req.out = None
        req.status = "released"
        self.in_use -= req.nbytes

    # ------------------------------------------------------------- statistics --
    def stats(self, since: float = 0.0) -> dict:
        """Latency percentiles (arrival to observed completion), the wait
        before launch and the launch-to-completion service time, over the
        requests that arrived at or after `since`."""
        span = [r for r in self.done if r.arrival >= since]
        lat = np.array([r.latency for r in span], np.float64)
        out = {"completed": int(lat.size), "rejected": len(self.rejected), "batches": self.batches,
               "peak_mem_bytes": int(self.peak_in_use)}
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
    A buffer is handed back only after the batch that wrote it completed and
    the client released it, so reuse on any stream is ordered."""

    def __init__(self, device):
        self.device = device
        self.free: Dict[Tuple[int, int], List[object]] = collections.defaultdict(list)
        self.allocated = 0

    def get(self, shape: Tuple[int, int]):
        lst = self.free.get(shape)
        if lst:
            return lst.pop()
        self.allocated += 1
        return torch.empty(shape, dtype=torch.float32, device=self.device)

    def put(self, bufs: Sequence[object]) -> None:
        for b in bufs:
            self.free[tuple(b.shape)].append(b)


class GraphExecutor(Executor):
    """Batches replayed as HIP graphs, each slot on its own stream of
    default priority.  Per slot and bucket there is one GraphBatch per
    capacity tier (e.g. 1, 4 and 16 frames): a batch runs on the smallest
    tier that holds it, so a lone request under light load does not pay for
    the launch grid of a full batch.  With `direct_single`, a lone request
    skips the graph (and its plan copy) and goes straight to ipb_complete_ws
    on the slot's stream, with a workspace resident per slot."""

    def __init__(self, slots: int = 2, max_batch: int = 16, device=None, default_params=None,
                 tiers: Optional[Sequence[int]] = None, direct_single: bool = True):
        from .api import Params
        self.direct_single = direct_single
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
        self.engines: Dict[Tuple[int, Hashable, int], object] = {}
        self.pool = BufferPool(self.device)

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
        return eng

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
            self.ws_bytes[slot] = need
        o = self.pool.get(r.shape)
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
        outs = [self.pool.get(r.shape) for r in reqs]
        ev = eng.run([r.frame for r in reqs], outs)
        return ev, outs

    def ready(self, handle) -> bool:
        return handle[0].query()

    def outputs(self, handle) -> List[object]:
        return handle[1]

    def recycle(self, outs: Sequence[object]) -> None:
        self.pool.put(outs)


class PerFrameExecutor(Executor):
    """The plain path: every request is one ipb_complete_ws call on a single
    stream as soon as it is admitted, so the device runs them in arrival
    order (one resident workspace serves them all).  `slots` bounds the
    requests in flight."""

    in_order = True

    def __init__(self, slots: int = 4096, device=None, default_params=None):
        from .api import Params
        self.slots = slots
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.default_params = default_params or Params()
        self.stream = torch.cuda.Stream(device=self.device)
        self.ws = None
        self.ws_bytes = 0
        self.cparams: Dict[Hashable, object] = {}
        self.pool = BufferPool(self.device)

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
            o = self.pool.get(r.shape)
            L.check(lib.ipb_complete_ws(ctypes.c_void_p(r.frame.data_ptr()), H, W, ctypes.byref(cp),
                                        ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                        self.ws_bytes, h), "ipb_complete_ws")
            outs.append(o)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev, outs

    def ready(self, handle) -> bool:
        return handle[0].query()

    def outputs(self, handle) -> List[object]:
        return handle[1]

    def recycle(self, outs: Sequence[object]) -> None:
        self.pool.put(outs)
