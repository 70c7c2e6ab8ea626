"""Benchmark of the depth-completion chain on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

Workloads (seeded synthetic LIDAR-shaped sparse depth maps, float32):
  c2 (default)  64 x 375x1242, 4-6 % valid, one batched launch per phase
  c1            one 352x1216 frame: per-call latency
  c3            128 frames of uneven sizes (H 256-512, W 768-2048)
  c4            16 x 1024x4096, 3 % valid, 1-120 m, offset 140
  c5            serving: Poisson arrivals at 500 / 2000 / 8000 frames/s of a
                size mix (and 16000 as an overload point), continuous batching
                against the plain per-frame path

One step = one batch through all nine stages.  Inputs are resident in HBM;
at least three buffer sets (input, output, workspace) are rotated so the
256 MB Infinity Cache cannot serve a step from the previous one.  The timed
batches of the batched workloads are spread over --streams streams (3 by
default), each buffer set bound to one of them and each stream on a
hardware queue of its own, so independent batches overlap; the same batches
on one stream are timed and reported too.  Prints
one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s and HBM GB/s at 375x1242 batched; p50/p99 latency under serving load"
HBM_PEAK_GBPS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # non-packed 32-bit VALU lane-operations
# launch steps of one batch (ipb_complete_planned phases 0..5) and the kernels each launches
PHASES = ["k_reset", "k_local_stream", "k_fill_scan+k_fill_tiles", "k_global_rows",
          "k_fill_cells+k_fill_dense+k_global_patched", "k_global_slow"]
# algorithmic HBM bytes per pixel: stage-1 input read + stage-4 map write (phase 1);
# stage-4 map read + output write (phase 2)
BYTES_PER_PX = {"k_local_stream": 8, "k_global_rows": 8}
CSRC = os.path.join(ROOT, "paper_1802_00036_amd", "csrc")
KERNEL_SOURCES = ("common.hpp", "networks.hpp", "median_net.hpp", "median_rows.hpp", "offsets.hpp", "kernels.hip",
                  "stream.hip",
                  "api.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2_batched.json")
PARAMS_TEXT = "diamond5 close5 fill7 extend fill31 median5 gauss5(binomial)"
WORKLOADS = {
    "c1": "one LIDAR-shaped sparse depth map, 352x1216 float32, 64 scan rows, 5 % valid, 1-80 m; per-call latency",
    "c2": "batch of 64 LIDAR-shaped sparse depth maps, 375x1242 float32, 64 scan rows, 4-6 % valid, 1-80 m; "
          "one batched launch per phase, tuned tiles, three batches in flight on three streams",
    "c3": "uneven batch of 128 LIDAR-shaped maps, H U{256..512} x W U{768..2048}, 32/64/128 scan rows, "
          "2-10 % valid; one batched launch per phase, tuned tiles, three batches in flight on three streams",
    "c4": "16 LIDAR-shaped maps of 1024x4096, 128 scan rows, 3 % valid, 1-120 m (offset 140), empty sky "
          "and occlusions; one batched launch per phase, tuned tiles, three batches in flight on three streams",
    "c5": "serving: Poisson arrivals at 500/2000/8000 frames/s, sizes 352x1216/375x1242/512x2048/1024x4096 "
          "(0.4/0.3/0.2/0.1), 2-10 % valid; device-resident inputs (no host transfer), continuous batching "
          "against one ipb_complete_ws per request on one stream",
}


# ------------------------------------------------------------ CPU baseline --

def _oracle_frame(task) -> float:
    import oracle
    from paper_1802_00036_amd import synth
    cfg, i = task
    f = synth.config_frame(cfg, i)
    p = oracle.Params(max_depth=140.0) if cfg == 4 else oracle.Params()
    t = time.perf_counter()
    oracle.complete_map(f.sparse, p)
    return time.perf_counter() - t


def cpu_baseline(cfg: int, n_frames: int) -> dict:
    """The CPU oracle over a bounded sample of the same workload (its first
    n frames), one frame per task over a process pool.  Runs before anything
    touches the GPU."""
    procs = max(1, min(16, os.cpu_count() or 1, n_frames))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        per = pool.map(_oracle_frame, [(cfg, i) for i in range(n_frames)])
    wall = time.perf_counter() - t0
    return {"value": round(n_frames / wall, 2), "unit": "frames/s", "cores": procs, "kind": "oracle",
            "sample": f"frames 0-{n_frames - 1} of the workload, all nine stages, {procs} processes; "
                      f"{sum(per):.1f} s of single-core oracle time ({sum(per) / n_frames:.3f} s/frame)"}


def _serve_frame(task):
    from paper_1802_00036_amd import synth
    s, i = task
    return synth.serve_frame(s, i).sparse


def serve_pool_host(per_size: int) -> dict:
    """Pre-generated frames of the serving mix (host), per size index."""
    from paper_1802_00036_amd import synth
    tasks = [(s, i) for s in range(len(synth.SERVE_SIZES)) for i in range(per_size)]
    ctx = mp.get_context("fork")
    with ctx.Pool(max(1, min(16, os.cpu_count() or 1))) as pool:
        maps = pool.map(_serve_frame, tasks, chunksize=4)
    out = {}
    for (s, _), m in zip(tasks, maps):
        out.setdefault(s, []).append(m)
    return out


# ---------------------------------------------------------------- GPU part --

def kernel_sha() -> str:
    """Hash of the library sources, to tell whether committed counter
    readings were taken on the current kernels."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_for(kernel: str, workload: str):
    """The kernel's entry in the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and this workload."""
    if workload != "c2":
        return None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("kernels", {}).get(kernel)


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled) or None."""
    k = profile_for(kernel, workload)
    return None if k is None else k.get("hbm_bytes_per_launch")


def valu_ceiling(kernel: str, workload: str, ms: float):
    """The kernel against the vector-ALU issue ceiling: lane-operations per
    launch (SQ_INSTS_VALU x 64 from the committed counter summary) over the
    launch duration measured here, against 256 CUs x 4 SIMD16 x 16 lanes x
    2.4 GHz = 39.3 T lane-ops/s (a wave64 instruction takes 4 cycles)."""
    k = profile_for(kernel, workload)
    if k is None or not k.get("valu_instr_per_launch"):
        return None
    ops = 64 * k["valu_instr_per_launch"]
    achieved = ops / (ms / 1e3) / 1e12
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 2), "peak": VALU_PEAK_TOPS,
            "unit": "T lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "lane_ops_per_launch": ops,
            "source": "SQ_INSTS_VALU from the committed counter summary, duration from this run"}


class Batches:
    """Rotating buffer sets of one batch (inputs, outputs, workspace, device
    plan), each bound to one of n_streams streams (all at the default
    priority, each on a hardware queue of its own).  Batches are independent,
    so batches on different streams may run at once; a set is only ever used
    on its own stream."""

    def __init__(self, host_maps, params, n_streams=1):
        import torch
        from paper_1802_00036_amd import _lib as L
        from paper_1802_00036_amd import api
        self.L, self.api, self.torch = L, api, torch
        self.lib = L.lib()
        self.params = params
        self.cp = params.to_c()
        self.dev = torch.device("cuda:0")
        self.n = len(host_maps)
        self.shapes = [m.shape for m in host_maps]
        # frames under 3 rows or columns take a launch step of their own (5);
        # a batch without one leaves it out (ipb_complete_planned phase -2)
        self.steps = list(range(len(PHASES)))
        if all(H >= 3 and W >= 3 for H, W in self.shapes):
            self.steps.remove(PHASES.index("k_global_slow"))
        self.px = sum(H * W for H, W in self.shapes)
        # streams from torch's pool share a few hardware queues, at times two
        # of them one queue, whose batches would then run one after the other
        self.streams = api.queue_streams(n_streams, self.dev)
        n_sets = n_streams * -(-3 // n_streams)        # at least three, a multiple of the streams
        self.sets = []
        for k in range(n_sets):
            ins = [torch.from_numpy(m).to(self.dev) for m in host_maps]
            outs = [torch.empty_like(t) for t in ins]
            arr = api.frames_array(ins, outs)
            nb = int(self.lib.ipb_batch_workspace_bytes(arr, self.n, ctypes.byref(self.cp)))
            ws = api._workspace(nb, self.dev)
            pb = int(self.lib.ipb_batch_plan_bytes(self.n))
            plan_h = ctypes.create_string_buffer(pb)
            L.check(self.lib.ipb_batch_plan(arr, self.n, ctypes.byref(self.cp), ctypes.c_void_p(ws.data_ptr()), nb,
                                            plan_h, pb), "ipb_batch_plan")
            n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
            self.lib.ipb_plan_totals(plan_h, ctypes.byref(n), ctypes.byref(lt), ctypes.byref(gt), ctypes.byref(cols))
            plan_d = torch.frombuffer(bytearray(plan_h.raw), dtype=torch.uint8).to(self.dev)
            s = self.streams[k % n_streams]
            self.sets.append(dict(ins=ins, outs=outs, ws=ws, plan=plan_d, lt=lt.value, gt=gt.value, cols=cols.value,
                                  stream=s))
        self.stream = self.streams[0]
        self.sh = ctypes.c_void_p(self.stream.cuda_stream)

    def run_phase(self, st, phase, stream=None):
        s = stream if stream is not None else st["stream"]
        self.L.check(self.lib.ipb_complete_planned(ctypes.c_void_p(st["plan"].data_ptr()), ctypes.byref(self.cp),
                                                   phase, st["lt"], st["gt"], st["cols"],
                                                   ctypes.c_void_p(s.cuda_stream)),
                     "ipb_complete_planned")

    def time_planned(self, steps, warmup):
        """Two timed passes of `steps` batches each.

        Serial: every batch on one stream, one after the other; the dominant
        kernel's mean duration comes from HIP events around it on that stream
        in the same steps (two events per step; the other launch steps run
        between them unbracketed).
        Streams: batch i on the stream of buffer set i mod sets, so batches
        on different streams overlap (one batch's small latency-bound steps
        and kernel tails run beside another's large kernels).  The time is
        from an event on the first stream, which the others wait for, to an
        event on it after it has waited for all of them.

        Per-step durations of every launch step come from a separate, untimed
        serial pass with events between all steps (those events add a few
        microseconds per step).  The steps are those the batch needs: the one
        of frames under 3 rows or columns only when the batch holds such a
        frame.  Returns the serial (ms per batch, dominant (name, ms)), the
        streams' ms per batch, the per-step durations and the wall time of
        the streams' pass."""
        torch = self.torch
        whole = -1 if PHASES.index("k_global_slow") in self.steps else -2
        for i in range(warmup):
            self.run_phase(self.sets[i % len(self.sets)], whole)
        torch.cuda.synchronize()
        # untimed serial pass: every launch step bracketed
        diag = max(5, min(steps, 50))
        ns = len(self.steps)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)] for _ in range(diag)]
        for i in range(diag):
            st = self.sets[i % len(self.sets)]
            for j, ph in enumerate(self.steps):
                evs[i][j].record(self.stream)
                self.run_phase(st, ph, self.stream)
            evs[i][ns].record(self.stream)
        torch.cuda.synchronize()
        k_ms = {name: 0.0 for name in PHASES}
        for j, ph in enumerate(self.steps):
            k_ms[PHASES[ph]] = sum(e[j].elapsed_time(e[j + 1]) for e in evs) / diag
        dom = max(BYTES_PER_PX, key=lambda k: k_ms[k])
        dph = PHASES.index(dom)
        # timed serial pass
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(self.stream)
        for i in range(steps):
            st = self.sets[i % len(self.sets)]
            for ph in self.steps:
                if ph == dph:
                    ev[i][0].record(self.stream)
                    self.run_phase(st, ph, self.stream)
                    ev[i][1].record(self.stream)
                else:
                    self.run_phase(st, ph, self.stream)
        t1.record(self.stream)
        torch.cuda.synchronize()
        serial_ms = t0.elapsed_time(t1) / steps
        dom_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        ref = [o.clone() for o in self.sets[0]["outs"]]
        # timed pass over the streams
        s0, others = self.streams[0], self.streams[1:]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t0.record(s0)
        for s in others:
            s.wait_event(t0)
        for i in range(steps):
            self.run_phase(self.sets[i % len(self.sets)], whole)
        for s in others:
            e = torch.cuda.Event()
            e.record(s)
            s0.wait_event(e)
        t1.record(s0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        if not all(torch.equal(a, b) for a, b in zip(ref, self.sets[0]["outs"])):
            raise RuntimeError("batches spread over streams gave other outputs than the serial pass")
        return (serial_ms, (dom, dom_ms)), t0.elapsed_time(t1) / steps, k_ms, wall

    def time_graph(self, steps, warmup, chain=True):
        """Mean ms per batch through GraphBatch (plan rewrite + one graph
        replay), one engine per buffer set, each on its own stream: chained
        (every batch after the previous one), or as a GraphPipeline (batch i
        on engine i mod engines, the engines' batches overlapping)."""
        torch = self.torch
        from paper_1802_00036_amd.batch import GraphBatch, GraphPipeline
        n = len(self.sets)
        if chain:
            engines = [GraphBatch(self.shapes, self.params, device=self.dev) for _ in self.sets]

            def submit(i, last):
                k = i % n
                # engines run on their own streams: chain them to keep batches in sequence
                if last is not None:
                    engines[k].stream.wait_event(last)
                return engines[k].run(self.sets[k]["ins"], self.sets[k]["outs"])
        else:
            pipe = GraphPipeline(self.shapes, self.params, engines=n, device=self.dev)
            engines = pipe.engines

            def submit(i, last):
                return pipe.run(self.sets[i % n]["ins"], self.sets[i % n]["outs"])   # set i mod n on engine i mod n
        last = None
        for i in range(max(warmup, 2 * n)):
            last = submit(i, last)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        last = None
        for i in range(steps):
            last = submit(i, last)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        return 1e3 * wall / steps, sum(e.replays for e in engines)

    def time_per_frame(self, reps):
        """Mean ms for the batch as one ipb_complete_ws call per frame, with
        the library's tiles for single frames (the batch's tuned tiles are
        chosen for whole batches)."""
        torch, api, L = self.torch, self.api, self.L
        st = self.sets[0]
        single = dataclasses.replace(self.params, tile_local=0, tile_global=0)
        cp = single.to_c()
        fws = api._workspace(max(api.workspace_bytes(H, W, single) for H, W in self.shapes), self.dev)
        fnb = fws.numel()

        def once():
            for i, (H, W) in enumerate(self.shapes):
                L.check(self.lib.ipb_complete_ws(ctypes.c_void_p(st["ins"][i].data_ptr()), H, W,
                                                 ctypes.byref(cp), ctypes.c_void_p(st["outs"][i].data_ptr()),
                                                 ctypes.c_void_p(fws.data_ptr()), fnb, self.sh), "ipb_complete_ws")
        for _ in range(2):
            once()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            once()
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps


def copy_probe_gbps(reps=20):
    """HBM bandwidth a plain streaming kernel attains here: torch.mul over
    256 MiB in and 256 MiB out, mean of `reps` event-timed launches."""
    import torch
    src_t = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst_t = torch.empty_like(src_t)
    for _ in range(3):
        torch.mul(src_t, 2.0, out=dst_t)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        torch.mul(src_t, 2.0, out=dst_t)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src_t, dst_t
    return round(2 * (256 << 20) / (ms / 1e3) / 1e9, 1)


def roofline(dom_timed, px, workload):
    dom, ms = dom_timed
    achieved = BYTES_PER_PX[dom] * px / (ms / 1e3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic_for(dom, workload),
            "launch_ms": round(ms, 5), "bytes_per_launch": BYTES_PER_PX[dom] * px}


def record(args, workload, value, unit, ms_step, extra, higher=True):
    rec = {
        "metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None if ms_step is None else round(ms_step, 5), "higher_is_better": higher,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS[workload], "id": workload, "params": PARAMS_TEXT},
    }
    rec.update(extra)
    rec["paper_context"] = ("90 frames/s on an Intel Core i7-7700K CPU (Table 1, Sec. IV), KITTI frames; "
                            "context only")
    print(json.dumps(rec), flush=True)


def bench_batch(args, workload, cpu, serve_host=None):
    import torch
    from paper_1802_00036_amd import api, synth
    cfg = int(workload[1])
    params = api.Params(max_depth=140.0) if cfg == 4 else api.Params()
    maps = [f.sparse for f in synth.config_frames(cfg)]
    extra = {}
    # tile shapes tuned for this batch, run as the timed pass runs it (batches
    # in flight on args.streams streams): the user cache's or the shipped
    # table's entry, else tuned here
    if args.tiles:
        tl, tg = (int(v) for v in args.tiles.split("/"))
        params = dataclasses.replace(params, tile_local=tl, tile_global=tg)
        extra["autotune"] = {"tile_local": tl, "tile_global": tg, "source": "--tiles"}
    elif not args.no_tune:
        from paper_1802_00036_amd import autotune
        probe = [torch.from_numpy(m).to("cuda:0") for m in maps]
        report = []
        params = autotune.tune(probe, params, reps=3, use_cache=not args.retune, report=report,
                               streams=args.streams)
        extra["autotune"] = {"tile_local": params.tile_local, "tile_global": params.tile_global,
                             "source": "tuned in this run" if report else "cached or shipped entry for this batch",
                             "candidates_us": [(r["phase"], r["tile"], None if r["us"] is None else round(r["us"], 1))
                                               for r in report]}
        del probe
    b = Batches(maps, params, n_streams=args.streams)
    (serial_ms, dom_timed), ms_step, k_ms, wall = b.time_planned(args.steps, args.warmup)
    fps = b.n / (ms_step / 1e3)
    rf = roofline(dom_timed, b.px, workload)
    rf["measured_in"] = "the serial timed pass: the kernel alone on the GPU"
    rf["copy_probe_gbps"] = copy_probe_gbps()
    rf["frac_of_copy_probe"] = round(rf["achieved"] / rf["copy_probe_gbps"], 4)
    extra.update({
        "config": None,
        "streams": args.streams,
        "serial_path": {"frames_per_s": round(b.n / (serial_ms / 1e3), 1), "ms_per_batch": round(serial_ms, 5),
                        "note": "the same batches on one stream, one after the other"},
        "roofline": rf,
        "valu_ceiling": valu_ceiling(dom_timed[0], workload, dom_timed[1]),
        "cpu_baseline": cpu,
        "hbm_gbps_algorithmic_pipeline": round(16 * b.px / (ms_step / 1e3) / 1e9, 1),
        "kernel_ms": {k: round(v, 5) for k, v in k_ms.items()},
        "kernel_ms_note": "untimed pass with HIP events between every launch step",
        "wall_s": round(wall, 3),
    })
    g_ms, replays = b.time_graph(max(10, args.steps // 2), 4)
    extra["graph_path"] = {"frames_per_s": round(b.n / (g_ms / 1e3), 1), "ms_per_batch": round(g_ms, 4),
                           "replays": replays, "note": "host clock around plan rewrite + graph replay, "
                                                       "batches one after another"}
    g_ms, replays = b.time_graph(max(10, args.steps // 2), 4, chain=False)
    extra["graph_path_overlapped"] = {"frames_per_s": round(b.n / (g_ms / 1e3), 1), "ms_per_batch": round(g_ms, 4),
                                      "replays": replays, "note": f"GraphPipeline of {len(b.sets)} engines on their own "
                                                                  "streams, batches overlapping"}
    if args.per_frame_steps > 0:
        pf_ms = b.time_per_frame(args.per_frame_steps)
        extra["per_frame_path"] = {"frames_per_s": round(b.n / (pf_ms / 1e3), 1), "ms_per_batch": round(pf_ms, 4)}
    if serve_host is not None:
        # the serving mix at a rate where batches form (8000 frames/s) and at
        # an overload point (16000), the batcher beside the plain per-frame
        # FIFO on the same arrival traces
        extra["serving"] = serving_runs(serve_host, rates=(8000, 16000), seconds=args.serve_seconds,
                                        modes=("batched", "per_frame"), warmup_s=0.5)
    cfgd = {"workload": WORKLOADS[workload], "id": workload, "frames": b.n, "pixels": b.px, "params": PARAMS_TEXT}
    if cfg in (2, 4):
        cfgd.update(H=b.shapes[0][0], W=b.shapes[0][1])
    extra["config"] = cfgd
    record(args, workload, round(fps, 1), "frames/s", ms_step, extra)


def bench_latency(args, cpu):
    import torch
    from paper_1802_00036_amd import api, synth
    from paper_1802_00036_amd.batch import GraphBatch
    m = synth.config_frames(1)[0].sparse
    x = torch.from_numpy(m).to("cuda:0")
    out = torch.empty_like(x)
    lat = {}
    for name in ("per_call", "graph"):
        if name == "graph":
            gb = GraphBatch([m.shape])
        times = []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            if name == "graph":
                gb.run([x], [out]).synchronize()
            else:
                api.complete(x, out=out)
                torch.cuda.synchronize()
            if i >= args.warmup:
                times.append(time.perf_counter() - t)
        times.sort()
        lat[name] = {"p50_ms": round(1e3 * times[len(times) // 2], 4),
                     "p99_ms": round(1e3 * times[min(len(times) - 1, int(0.99 * len(times)))], 4)}
    # the value: one ipb_complete_ws call per frame (the graph path adds the
    # host's plan rewrite and the plan copy)
    record(args, "c1", lat["per_call"]["p50_ms"], "ms (p50 latency, host clock)", lat["per_call"]["p50_ms"],
           {"latency": lat, "cpu_baseline": cpu}, higher=False)


def serving_runs(host_pool, rates, seconds, modes=("batched", "per_frame"), warmup_s=1.0):
    import numpy as np
    import torch
    from paper_1802_00036_amd import api, serve, synth
    dev = torch.device("cuda:0")
    pool = {s: [torch.from_numpy(m).to(dev) for m in maps] for s, maps in host_pool.items()}
    torch.cuda.synchronize()
    p140 = api.Params(max_depth=140.0)
    big = [i for i, (H, _) in enumerate(synth.SERVE_SIZES) if H >= 1024]
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(min(8 << 30, free // 4))
    out = {}
    for mode in modes:
        for rate in rates:
            n = int(rate * (seconds + warmup_s))
            arrivals, sizes = synth.poisson_arrivals(rate, n)
            frames = [pool[int(s)][i % len(pool[int(s)])] for i, s in enumerate(sizes)]
            params = [p140 if int(s) in big else None for s in sizes]
            # the pool's frames were made and synchronised before the trace
            # starts: launches need not wait for the stream they came from
            if mode == "batched":
                ex = serve.GraphExecutor(slots=3, max_batch=16, order_inputs=False)
                ex.warm([((serve.default_bucket(synth.SERVE_SIZES[s]), serve._params_key(p140 if s in big else None)),
                          p140 if s in big else None) for s in range(len(synth.SERVE_SIZES))])
                srv = serve.Server(ex, mem_budget=budget, max_batch=16, keep_outputs=False)
            else:
                ex = serve.PerFrameExecutor(order_inputs=False)
                srv = serve.Server(ex, mem_budget=budget, max_batch=1, keep_outputs=False)
                for s in range(len(synth.SERVE_SIZES)):
                    api.complete(pool[s][0], p140 if s in big else None)
            torch.cuda.synchronize()
            st = serve.run_trace(srv, frames, arrivals, params, warmup=warmup_s)
            st = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
            st["offered_fps"] = rate
            st["requests"] = n
            out[f"{mode}@{rate}"] = st
            print(f"[serve] {mode} {rate}/s: {st}", file=sys.stderr, flush=True)
            del srv, ex
            torch.cuda.synchronize()
    return out


def bench_serving(args, host_pool):
    res = serving_runs(host_pool, rates=(500, 2000, 8000, 16000), seconds=args.serve_seconds)
    top = res.get("batched@2000", {})
    record(args, "c5", top.get("p99_ms"), "ms (p99 latency at 2000 frames/s offered)", None,
           {"serving": res, "pool_frames_per_size": args.serve_pool, "cpu_baseline": None}, higher=False)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-frame-steps", type=int, default=10)
    ap.add_argument("--streams", type=int, default=3,
                    help="batched workloads: streams the timed batches are spread over (buffer sets are bound "
                         "to streams; batches on different streams overlap)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-pool", type=int, default=64, help="pre-generated frames per size for serving")
    ap.add_argument("--no-serving", action="store_true", help="c2: skip the serving summary")
    ap.add_argument("--no-tune", action="store_true", help="default tile shapes instead of the autotuner's")
    ap.add_argument("--tiles", default=None, metavar="L/G",
                    help="batched workloads: phase-1/phase-2 tile ids to run instead of the autotuner's")
    ap.add_argument("--retune", action="store_true",
                    help="tune now instead of taking the cached or shipped entry for the batch")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain kernel reading and writing 256 MiB (calibrates rocprofv3 "
                         "FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); frames are independent, so a "
              "multi-GPU run would shard whole frames across devices with no exchange.", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    # host work that forks runs before the GPU is touched
    n_cpu = {"c1": 1, "c2": 64, "c3": 128, "c4": 16}.get(wl)
    cpu = None if (args.no_cpu_baseline or n_cpu is None) else cpu_baseline(int(wl[1]), n_cpu)
    host_pool = None
    if wl == "c5" or (wl == "c2" and not args.no_serving):
        host_pool = serve_pool_host(args.serve_pool)

    import torch
    torch.cuda.set_device(0)
    if wl == "c1":
        bench_latency(args, cpu)
    elif wl == "c5":
        bench_serving(args, host_pool)
    else:
        bench_batch(args, wl, cpu, host_pool)

    if args.copy_probe:
        # a plain streaming kernel that reads 256 MiB and writes 256 MiB
        src_t = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            torch.mul(src_t, 2.0, out=dst_t)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
