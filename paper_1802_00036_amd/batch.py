"""Batches of frames of uneven sizes through one captured launch sequence.

A `GraphBatch` owns, for a stated capacity, a device workspace, a device copy
of the launch plan and two pinned host plans.  The first run on each pinned
plan executes eagerly and captures the same work into a HIP graph: a copy of
the pinned plan into device memory, then every kernel of the chain with grids
derived from the capacity (ipb_complete_planned).  Later runs only rewrite the
pinned plan (frame pointers and sizes) and replay the graph, so any batch
within the capacity is one graph launch.  The graph leaves out the launch step
for frames under 3 rows or columns; a batch that holds such a frame runs
eagerly with every step instead.  The two pinned plans alternate: the
host rewrites a plan only after the replay that last read it has finished,
so batch k+1 can be queued while batch k runs.

Frames are independent (Sec. II: each map is completed from its own points);
the plan only tells the kernels where each frame's tiles start.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .api import Params, _check_map, _frames_array, _stream_handle, _workspace, queue_streams

Shape = Tuple[int, int]
# the library's automatic tile rule, in waves (MI355X: 256 CUs x 4 SIMDs)
AUTO_LOCAL32, AUTO_LOCAL16, AUTO_LOCAL8, AUTO_GLOBAL = 2048, 1024, 512, 4096


def _tile_counts(p: L.CParams, shapes: Sequence[Shape]) -> Tuple[int, int, int]:
    """Tiles of phase 1, tiles of phase 2 and columns of a list of shapes."""
    lib = L.lib()
    rows, cols = ctypes.c_int(), ctypes.c_int()
    out = []
    for phase, tid in ((1, p.tile_local), (2, p.tile_global)):
        L.check(lib.ipb_tile_shape(phase, tid, ctypes.byref(rows), ctypes.byref(cols)), "ipb_tile_shape")
        out.append(sum(-(-H // rows.value) * -(-W // cols.value) for H, W in shapes))
    return out[0], out[1], sum(W for _, W in shapes)


def _placeholder_bytes(shapes: Sequence[Shape], params: Params) -> int:
    """ipb_batch_workspace_bytes for frames of these shapes (0: invalid or
    unsupported).  The call reads only sizes; the descriptors carry distinct
    placeholder addresses (every frame in place) that are never
    dereferenced."""
    arr = (L.CFrame * len(shapes))()
    addr = 1 << 40
    for i, (H, W) in enumerate(shapes):
        arr[i].in_ = addr
        arr[i].out = addr
        arr[i].H, arr[i].W = H, W
        addr += (4 * H * W + 255) // 256 * 256
    p = params.to_c()
    return int(L.lib().ipb_batch_workspace_bytes(arr, len(shapes), ctypes.byref(p)))


def shapes_workspace_bytes(shapes: Sequence[Shape], params: Optional[Params] = None) -> int:
    """ipb_batch_workspace_bytes for frames of these shapes."""
    nb = _placeholder_bytes(shapes, params or Params())
    if nb == 0:
        L.check(L.IPB_ERR_INVALID_ARG, "ipb_batch_workspace_bytes")
    return nb


def auto_tiles(params: Params, shapes: Sequence[Shape]) -> Params:
    """The tiles the library picks for a call that sees frames of these
    shapes, as explicit ids (tile id 0 only): phase-1 tiles of 32 rows when
    64-row ones would give the GPU fewer than two waves per SIMD, of 16 rows
    when 32-row ones would give fewer than one, of 8 rows when 16-row ones
    would give fewer than half; phase-2 tiles (the default chain only) of the
    tallest of 32, 16 and 8 rows that gives at least four.  Only tiles the
    chain supports."""
    def count(p: Params, phase: int, tid: int) -> int:
        q = dataclasses.replace(p, **{"tile_local" if phase == 1 else "tile_global": tid})
        return _tile_counts(q.to_c(), shapes)[phase - 1]
    if params.tile_local == 0 and count(params, 1, 0) < AUTO_LOCAL32:
        tid = 7 if count(params, 1, 7) >= AUTO_LOCAL16 else 8 if count(params, 1, 8) >= AUTO_LOCAL8 else 9
        small = dataclasses.replace(params, tile_local=tid)
        if _placeholder_bytes(shapes, small) > 0:
            params = small
    if params.tile_global == 0 and count(params, 2, 0) < AUTO_GLOBAL:
        small = dataclasses.replace(params, tile_global=8 if count(params, 2, 8) >= AUTO_GLOBAL else 9)
        if _placeholder_bytes(shapes, small) > 0:
            params = small
    return params


class GraphBatch:
    """Graph-replayed batched completion for batches up to a capacity.

    capacity: the shapes of the largest batch this object must run.  A batch
    fits if it has no more frames, its workspace is no larger and its tile and
    column totals are no larger than those of the capacity.
    """

    def __init__(self, capacity: Sequence[Shape], params: Optional[Params] = None,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None,
                 use_graph: bool = True):
        if not capacity:
            raise ValueError("capacity must name at least one frame shape")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.capacity = [tuple(int(v) for v in s) for s in capacity]
        params = params or Params()
        params = auto_tiles(params, self.capacity)   # the plan and the captured launch share them
        self.params = params
        self.cp = self.params.to_c()
        self.max_frames = len(self.capacity)
        self.max_lt, self.max_gt, self.max_cols = _tile_counts(self.cp, self.capacity)
        self.ws_bytes = shapes_workspace_bytes(self.capacity, self.params)
        self.plan_bytes = int(L.lib().ipb_batch_plan_bytes(self.max_frames))
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.ws = _workspace(self.ws_bytes, self.device)
        self.plan_dev = _workspace(self.plan_bytes, self.device)
        self.plan_host = [torch.empty(self.plan_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.use_graph = use_graph
        self.graphs: List[Optional[torch.cuda.CUDAGraph]] = [None, None]
        self.done = [None, None]          # event after the last run that read plan_host[k]
        self.turn = 0
        self.replays = 0

    @classmethod
    def for_batch(cls, frames: Sequence[torch.Tensor], params: Optional[Params] = None, **kw) -> "GraphBatch":
        return cls([tuple(f.shape) for f in frames], params, device=frames[0].device, **kw)

    def fits(self, shapes: Sequence[Shape]) -> bool:
        if not shapes or len(shapes) > self.max_frames:
            return False
        lt, gt, cols = _tile_counts(self.cp, shapes)
        if lt > self.max_lt or gt > self.max_gt or cols > self.max_cols:
            return False
        return shapes_workspace_bytes(shapes, self.params) <= self.ws_bytes

    def _enqueue(self, k: int, phase: int) -> None:
        self.plan_dev.copy_(self.plan_host[k], non_blocking=True)
        st = L.lib().ipb_complete_planned(ctypes.c_void_p(self.plan_dev.data_ptr()), ctypes.byref(self.cp), phase,
                                          self.max_lt, self.max_gt, self.max_cols,
                                          _stream_handle(torch.cuda.current_stream()))
        L.check(st, "ipb_complete_planned")

    def run(self, frames: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None) -> torch.cuda.Event:
        """Queue the completion of `frames` into `outs` (new tensors if None)
        on this object's stream; returns the event that marks its end.  The
        caller keeps inputs and outputs alive until then, and makes the
        stream wait for whatever produced the inputs."""
        frames = list(frames)
        if outs is None:
            with torch.cuda.stream(self.stream):
                outs = [torch.empty_like(f) for f in frames]
        outs = list(outs)
        if not frames or len(frames) > self.max_frames:
            raise ValueError(f"batch of {len(frames)} frames; capacity {self.max_frames}")
        arr, side = _frames_array(frames, outs)
        k = self.turn
        self.turn ^= 1
        if self.done[k] is not None:
            self.done[k].synchronize()           # the run that last read plan_host[k]
        host = self.plan_host[k]
        st = L.lib().ipb_batch_plan(arr, len(frames), ctypes.byref(self.cp), ctypes.c_void_p(self.ws.data_ptr()),
                                    self.ws_bytes, ctypes.c_void_p(host.data_ptr()), self.plan_bytes)
        L.check(st, "ipb_batch_plan")
        n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
        L.check(L.lib().ipb_plan_totals(ctypes.c_void_p(host.data_ptr()), ctypes.byref(n), ctypes.byref(lt),
                                        ctypes.byref(gt), ctypes.byref(cols)), "ipb_plan_totals")
        if lt.value > self.max_lt or gt.value > self.max_gt or cols.value > self.max_cols:
            raise ValueError("batch exceeds the tile or column totals of the capacity")
        # the captured launch leaves out the step for frames under 3 rows or
        # columns (planned phase -2); a batch holding such a frame runs
        # eagerly with every step
        tiny = side < 3
        with torch.cuda.stream(self.stream):
            if not self.use_graph or tiny:
                self._enqueue(k, -1)
            elif self.graphs[k] is None:
                self._enqueue(k, -2)             # first run: eager, then capture the same work
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=self.stream):
                    self._enqueue(k, -2)
                self.graphs[k] = g
            else:
                self.graphs[k].replay()
                self.replays += 1
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.done[k] = ev
        self._outs = outs
        return ev

    def __call__(self, frames: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None
                 ) -> List[torch.Tensor]:
        """Run and make the current stream wait for the result."""
        for f in frames:
            _check_map(f, "frame")
        self.stream.wait_stream(torch.cuda.current_stream())
        ev = self.run(frames, outs)
        torch.cuda.current_stream().wait_event(ev)
        return self._outs


class GraphPipeline:
    """GraphBatch engines of one capacity, each on its own stream (all at the
    default priority, each on a hardware queue of its own: queue_streams),
    taking batches in turn.  Frames of different batches
    share nothing, so up to `engines` batches run on the GPU at once: one
    batch's short latency-bound launch steps and kernel tails overlap the
    large kernels of the others, which carries more frames per second than
    one engine whose batches run one after another."""

    def __init__(self, capacity: Sequence[Shape], params: Optional[Params] = None, engines: int = 3,
                 device: Optional[torch.device] = None, use_graph: bool = True):
        if engines < 1:
            raise ValueError("a pipeline needs at least one engine")
        streams = queue_streams(engines, device)
        self.engines = [GraphBatch(capacity, params, device=device, stream=s, use_graph=use_graph) for s in streams]
        self.turn = 0

    def next_stream(self) -> torch.cuda.Stream:
        """The stream the next batch runs on: make it wait for whatever
        produces that batch's inputs."""
        return self.engines[self.turn].stream

    def run(self, frames: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None) -> torch.cuda.Event:
        """Queue `frames` on the next engine (GraphBatch.run); returns the
        event that marks the batch's end.  The caller keeps inputs and
        outputs alive until then."""
        e = self.engines[self.turn]
        self.turn = (self.turn + 1) % len(self.engines)
        return e.run(frames, outs)
