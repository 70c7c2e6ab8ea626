"""Tile-shape autotuner for batched completion.

The library offers several tile shapes per phase (ipb_tile_shape): streaming
one-wave tiles of different heights and LDS tiles of different sizes.  Which
is fastest depends on the frame sizes (ragged edges, number of tiles per
launch against the 256 compute units) and on the parameters (halo widths).
`tune` times every supported shape on the caller's own frames, one phase at a
time (phase-1 shape first with the automatic phase-2 shape, then phase-2
shapes with the winner), and returns the parameters with the fastest pair.

Results are cached in a JSON file keyed by device, parameters and a coarse
signature of the batch (frame count, pixel total and median size, each
rounded), so one tuning serves every batch of the same kind.  The cache path
is $IPB_TUNE_CACHE, else ~/.cache/ipb/tune.json; tuning never changes
results, only speed (every tile shape is bit-exact against the same
definition).
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
from .api import Params, _stream_handle, _workspace, frames_array


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
    props = torch.cuda.get_device_properties(device)
    return f"{props.name}-{getattr(props, 'gcnArchName', '')}-{props.multi_processor_count}"


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


def candidate_ids(phase: int) -> List[int]:
    return list(range(1, int(L.lib().ipb_tile_count(phase)) + 1))


def tune(frames: Sequence[torch.Tensor], params: Optional[Params] = None, reps: int = 5,
         use_cache: bool = True, report: Optional[list] = None) -> Params:
    """Parameters with the fastest tile shapes for batches like `frames`
    (outputs and results are unchanged by the choice)."""
    p0 = params or Params()
    frames = list(frames)
    if not frames:
        return p0
    shapes = [tuple(f.shape) for f in frames]
    key = "|".join((device_signature(frames[0].device), params_signature(p0), batch_signature(shapes)))
    path = cache_path()
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            return dataclasses.replace(p0, tile_local=int(hit["tile_local"]), tile_global=int(hit["tile_global"]))
    stream = torch.cuda.Stream(device=frames[0].device)
    with torch.cuda.stream(stream):
        outs = [torch.empty_like(f) for f in frames]
    stream.wait_stream(torch.cuda.current_stream())
    timer = _Timer(frames, outs, stream)
    best_l, t_l = None, None
    for tl in candidate_ids(1):
        t = timer.time_us(dataclasses.replace(p0, tile_local=tl, tile_global=0), phases=(1, 2), reps=reps)
        if report is not None:
            report.append({"phase": 1, "tile": tl, "us": t})
        if t is not None and (t_l is None or t < t_l):
            best_l, t_l = tl, t
    best_g, t_g = None, None
    for tg in candidate_ids(2):
        t = timer.time_us(dataclasses.replace(p0, tile_local=best_l or 0, tile_global=tg), phases=(3, 4, 5),
                          reps=reps)
        if report is not None:
            report.append({"phase": 2, "tile": tg, "us": t})
        if t is not None and (t_g is None or t < t_g):
            best_g, t_g = tg, t
    tuned = dataclasses.replace(p0, tile_local=best_l or 0, tile_global=best_g or 0)
    if use_cache:
        _store_cache(path, key, {"tile_local": tuned.tile_local, "tile_global": tuned.tile_global,
                                 "us_local": t_l, "us_global": t_g})
    return tuned
