"""Tile-shape autotuner for batched completion.

The library offers several tile shapes per phase (ipb_tile_shape): streaming
one-wave tiles of different heights and LDS tiles of different sizes.  Which
is fastest depends on the frame sizes (ragged edges, number of tiles per
launch against the 256 compute units) and on the parameters (halo widths).
`tune` times every supported shape on the caller's own frames, one phase at a
time (phase-1 shape first with the automatic phase-2 shape, then phase-2
shapes with the winner), and returns the parameters with the fastest pair.
A caller that keeps several batches in flight on separate streams asks for
that (streams > 1): the three fastest shapes of each phase are then paired
and each pair is timed as whole batches spread over the streams, because
there a shape that issues fewer instructions (taller tiles, less halo) can
win although it fills the GPU less when it runs alone.

Results are cached in a JSON file keyed by device, parameters and a coarse
signature of the batch (frame count, pixel total and median size, each
rounded), so one tuning serves every batch of the same kind.  The cache path
is $IPB_TUNE_CACHE, else ~/.cache/ipb/tune.json.  A table of such entries
measured on MI355X for the benchmark batches ships beside this module
(tuned_mi355x.json, written by `python -m paper_1802_00036_amd.autotune`);
it is read when the user cache has no entry.  Tuning never changes results,
only speed (every tile shape is bit-exact against the same definition).
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .api import Params, _stream_handle, _workspace, frames_array, queue_streams


SHIPPED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def cache_path() -> str:
    return os.environ.get("IPB_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ipb", "tune.json")


def _round_log2(v: float, steps: int = 2) -> float:
    """v rounded to a grid of 2^(1/steps)."""
    if v <= 0:
        return 0.0
    return round(2.0 ** (round(math.log2(v) * steps) / steps), 3)


def batch_signature(shapes: Sequence[Tuple[int, int]]) -> str:
    n = len(shapes)
    px = sum(H * W for H, W in shapes)
    hs = sorted(H for H, _ in shapes)
    ws = sorted(W for _, W in shapes)
    return f"n{_round_log2(n)}-px{_round_log2(px)}-h{_round_log2(hs[n // 2], 4)}-w{_round_log2(ws[n // 2], 4)}"


def params_signature(p: Params) -> str:
    d = dataclasses.asdict(p)
    d.pop("tile_local")
    d.pop("tile_global")
    return ",".join(f"{k}={d[k]}" for k in sorted(d))


def device_signature(device: torch.device) -> str:
    """Architecture and compute-unit count (the marketing name is left out:
    the runtime reports a generic one when its name table is missing)."""
    props = torch.cuda.get_device_properties(device)
    return f"{getattr(props, 'gcnArchName', '')}-{props.multi_processor_count}"


def _load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, key: str, entry: dict) -> None:
    data = _load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


class _Timer:
    """Times ipb_complete_planned for one parameter set on fixed frames."""

    def __init__(self, frames: Sequence[torch.Tensor], outs: Sequence[torch.Tensor], stream: torch.cuda.Stream):
        self.frames, self.outs, self.stream = list(frames), list(outs), stream
        self.arr = frames_array(self.frames, self.outs)
        self.n = len(self.frames)
        self.plan_bytes = int(L.lib().ipb_batch_plan_bytes(self.n))
        self.host = torch.empty(self.plan_bytes, dtype=torch.uint8, pin_memory=True)
        self.dev = torch.empty(self.plan_bytes + 256, dtype=torch.uint8, device=self.frames[0].device)

    def time_us(self, p: Params, phases: Sequence[int], reps: int) -> Optional[float]:
        """Mean microseconds of the given launch steps, or None if the
        parameters are unsupported."""
        cp = p.to_c()
        lib = L.lib()
        ws_bytes = int(lib.ipb_batch_workspace_bytes(self.arr, self.n, ctypes.byref(cp)))
        if ws_bytes == 0:
            return None
        ws = _workspace(ws_bytes, self.frames[0].device)
        st = lib.ipb_batch_plan(self.arr, self.n, ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                                ctypes.c_void_p(self.host.data_ptr()), self.plan_bytes)
        if st == L.IPB_ERR_UNSUPPORTED:
            return None
        L.check(st, "ipb_batch_plan")
        n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
        lib.ipb_plan_totals(ctypes.c_void_p(self.host.data_ptr()), ctypes.byref(n), ctypes.byref(lt),
                            ctypes.byref(gt), ctypes.byref(cols))
        dev = self.dev[(-self.dev.data_ptr()) % 256:][:self.plan_bytes]
        s = self.stream
        with torch.cuda.stream(s):
            dev.copy_(self.host, non_blocking=True)
            h = _stream_handle(s)

            def step(phase):
                L.check(lib.ipb_complete_planned(ctypes.c_void_p(dev.data_ptr()), ctypes.byref(cp), phase,
                                                 lt.value, gt.value, cols.value, h), "ipb_complete_planned")

            total = 0.0
            for r in range(reps + 1):
                for ph in range(6):
                    if ph in phases:
                        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        a.record(s)
                        step(ph)
                        b.record(s)
                        b.synchronize()
                        if r > 0:                   # the first repetition warms up
                            total += a.elapsed_time(b) * 1e3
                    else:
                        step(ph)
            s.synchronize()
        return total / reps

    def throughput_us(self, p: Params, streams: int, reps: int) -> Optional[float]:
        """Microseconds per batch with `streams` batches in flight, one per
        stream (each with its own inputs, outputs, workspace and plan, as
        independent batches have), or None if the parameters are
        unsupported."""
        cp = p.to_c()
        lib = L.lib()
        dev0 = self.frames[0].device
        lanes = []
        # each batch on a hardware queue of its own: streams from torch's pool
        # put two batches on one queue now and then, which reads some 15 %
        # slow and ranks pairs by where their streams landed
        lane_streams = queue_streams(streams, dev0)
        for k in range(streams):
            ins = [f.clone() for f in self.frames] if k else self.frames
            outs = [torch.empty_like(f) for f in self.frames] if k else self.outs
            arr = frames_array(ins, outs)
            ws_bytes = int(lib.ipb_batch_workspace_bytes(arr, self.n, ctypes.byref(cp)))
            if ws_bytes == 0:
                return None
            ws = _workspace(ws_bytes, dev0)
            host = torch.empty(self.plan_bytes, dtype=torch.uint8, pin_memory=True)
            st = lib.ipb_batch_plan(arr, self.n, ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                                    ctypes.c_void_p(host.data_ptr()), self.plan_bytes)
            if st == L.IPB_ERR_UNSUPPORTED:
                return None
            L.check(st, "ipb_batch_plan")
            n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
            lib.ipb_plan_totals(ctypes.c_void_p(host.data_ptr()), ctypes.byref(n), ctypes.byref(lt),
                                ctypes.byref(gt), ctypes.byref(cols))
            s = lane_streams[k]
            dev = torch.empty(self.plan_bytes, dtype=torch.uint8, device=dev0)
            with torch.cuda.stream(s):
                dev.copy_(host, non_blocking=True)
            lanes.append((s, dev, host, outs, ws, lt.value, gt.value, cols.value, ins))

        # every launch step the batch needs: the one for frames under 3 rows
        # or columns only when it holds such a frame (as ipb_complete_batch)
        whole = -1 if any(min(f.shape) < 3 for f in self.frames) else -2

        def launch(lane):
            s, dev, _, _, _, lt, gt, cols, _ = lane
            L.check(lib.ipb_complete_planned(ctypes.c_void_p(dev.data_ptr()), ctypes.byref(cp), whole, lt, gt, cols,
                                             _stream_handle(s)), "ipb_complete_planned")

        torch.cuda.synchronize(dev0)               # the clones and plan copies
        for lane in lanes:                         # warm-up
            launch(lane)
        torch.cuda.synchronize(dev0)
        s0 = lanes[0][0]
        # the least of three timed passes: batches in flight vary by several
        # percent from pass to pass, and one pass would rank pairs by noise
        best = None
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s0)
            for lane in lanes[1:]:
                lane[0].wait_event(a)
            for _ in range(reps):
                for lane in lanes:
                    launch(lane)
            for lane in lanes[1:]:
                e = torch.cuda.Event()
                e.record(lane[0])
                s0.wait_event(e)
            b.record(s0)
            b.synchronize()
            torch.cuda.synchronize(dev0)
            us = a.elapsed_time(b) * 1e3 / (reps * streams)
            best = us if best is None else min(best, us)
        return best


def tune_key(frames: Sequence[torch.Tensor], params: Params, streams: int = 1) -> str:
    """Cache key of a batch: device, parameters, batch signature (and the
    stream count when batches run in flight)."""
    shapes = [tuple(f.shape) for f in frames]
    key = "|".join((device_signature(frames[0].device), params_signature(params), batch_signature(shapes)))
    return key + (f"|streams{streams}" if streams > 1 else "")


def lookup(frames: Sequence[torch.Tensor], params: Optional[Params] = None, streams: int = 1,
           user_cache: bool = True, shipped: bool = True) -> Optional[Params]:
    """The cached tiles for batches like `frames` without timing anything:
    the user cache's entry, else (shipped) the package table's; None if
    neither has one."""
    p0 = params or Params()
    frames = list(frames)
    if not frames:
        return None
    key = tune_key(frames, p0, streams)
    hit = _load_cache(cache_path()).get(key) if user_cache else None
    if hit is None and shipped:
        hit = _load_cache(SHIPPED_TABLE).get(key)
    if not hit:
        return None
    return dataclasses.replace(p0, tile_local=int(hit["tile_local"]), tile_global=int(hit["tile_global"]))


def candidate_ids(phase: int) -> List[int]:
    return list(range(1, int(L.lib().ipb_tile_count(phase)) + 1))


def tune(frames: Sequence[torch.Tensor], params: Optional[Params] = None, reps: int = 5,
         use_cache: bool = True, report: Optional[list] = None, streams: int = 1,
         use_shipped: bool = True) -> Params:
    """Parameters with the fastest tile shapes for batches like `frames`
    (outputs and results are unchanged by the choice), run one at a time
    (streams = 1) or `streams` batches in flight on as many streams.
    use_cache: read (and write) the user cache; use_shipped: also read the
    package's table when the user cache has no entry."""
    p0 = params or Params()
    frames = list(frames)
    if not frames:
        return p0
    key = tune_key(frames, p0, streams)
    path = cache_path()
    if use_cache:
        hit = lookup(frames, p0, streams, user_cache=True, shipped=use_shipped)
        if hit is not None:
            return hit
    stream = torch.cuda.Stream(device=frames[0].device)
    with torch.cuda.stream(stream):
        outs = [torch.empty_like(f) for f in frames]
    stream.wait_stream(torch.cuda.current_stream())
    timer = _Timer(frames, outs, stream)
    times_l = {}
    for tl in candidate_ids(1):
        t = timer.time_us(dataclasses.replace(p0, tile_local=tl, tile_global=0), phases=(1, 2), reps=reps)
        if report is not None:
            report.append({"phase": 1, "tile": tl, "us": t})
        if t is not None:
            times_l[tl] = t
    best_l = min(times_l, key=times_l.get) if times_l else None
    times_g = {}
    for tg in candidate_ids(2):
        t = timer.time_us(dataclasses.replace(p0, tile_local=best_l or 0, tile_global=tg), phases=(3, 4, 5),
                          reps=reps)
        if report is not None:
            report.append({"phase": 2, "tile": tg, "us": t})
        if t is not None:
            times_g[tg] = t
    best_g = min(times_g, key=times_g.get) if times_g else None
    entry = {"us_local": times_l.get(best_l), "us_global": times_g.get(best_g)}
    if streams > 1 and times_l and times_g:
        top_l = sorted(times_l, key=times_l.get)[:3]
        top_g = sorted(times_g, key=times_g.get)[:3]
        pair_us = {}
        for tl in top_l:
            for tg in top_g:
                t = timer.throughput_us(dataclasses.replace(p0, tile_local=tl, tile_global=tg), streams, reps)
                if report is not None:
                    report.append({"phase": f"{streams} streams", "tile": f"{tl}/{tg}", "us": t})
                if t is not None:
                    pair_us[(tl, tg)] = t
        if pair_us:
            # pairs within 1.5 % of the best are a tie (repeated timings of a
            # pair agree within about 1 %); of those, the one fastest with a
            # batch alone on the GPU
            fastest = min(pair_us.values())
            ties = [k for k, t in pair_us.items() if t <= 1.015 * fastest]
            best_l, best_g = min(ties, key=lambda k: times_l[k[0]] + times_g[k[1]])
            entry = {"us_per_batch": pair_us[(best_l, best_g)], "streams": streams}
    tuned = dataclasses.replace(p0, tile_local=best_l or 0, tile_global=best_g or 0)
    if use_cache:
        _store_cache(path, key, {"tile_local": tuned.tile_local, "tile_global": tuned.tile_global, **entry})
    return tuned


def _write_table(path: str, streams: int, reps: int) -> None:
    """Tune the benchmark batches (synth workloads 2, 3 and 4) for `streams`
    batches in flight and write their entries to `path`."""
    from . import synth
    table = {}
    for cfg in (2, 3, 4):
        frames = [torch.from_numpy(f.sparse).to("cuda:0") for f in synth.config_frames(cfg)]
        p0 = Params(max_depth=140.0) if cfg == 4 else Params()
        os.environ["IPB_TUNE_CACHE"] = path + ".tmp"
        report: list = []
        tuned = tune(frames, p0, reps=reps, use_cache=True, report=report, streams=streams, use_shipped=False)
        for r in report:
            print(f"  {r['phase']}: tile {r['tile']}: {r['us']} us", flush=True)
        entries = _load_cache(path + ".tmp")
        table.update(entries)
        print(f"workload {cfg}: tiles {tuned.tile_local}/{tuned.tile_global}", flush=True)
        del frames
    if os.path.exists(path + ".tmp"):
        os.remove(path + ".tmp")
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="write the shipped tuning table")
    ap.add_argument("--out", default=SHIPPED_TABLE)
    ap.add_argument("--streams", type=int, default=3)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    _write_table(a.out, a.streams, a.reps)
