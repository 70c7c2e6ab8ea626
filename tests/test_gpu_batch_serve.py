"""GPU tests of the batch engine (graph capture and replay), the tile
autotuner and the serving loop, all through the C ABI: every result must be
bit-identical to the same frame completed alone, which in turn equals the
oracle (checked on a sample)."""
import dataclasses
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1802_00036_amd import _lib as L
from paper_1802_00036_amd import api, autotune, batch, serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def bits(t):
    return np.ascontiguousarray(t.detach().cpu().numpy()).view(np.uint32)


def ntiles(phase):
    return int(L.lib().ipb_tile_count(phase))


def lidar(H, W, seed, density=0.05):
    return torch.from_numpy(synth.lidar_frame(H, W, seed=seed, n_rows=min(64, H), density=density).sparse).to(DEV)


def test_graph_replays_match_eager_across_batches():
    rng = np.random.default_rng(21)
    cap = [(300, 700)] * 6
    gb = batch.GraphBatch(cap, device=torch.device(DEV))
    batches = []
    for b in range(5):
        n = int(rng.integers(1, 7))
        shapes = [(int(rng.integers(1, 301)), int(rng.integers(1, 701))) for _ in range(n)]
        if b == 2:
            shapes = [(1, 1), (2, 5), (300, 700)][:n] or [(1, 1)]
        batches.append([lidar(H, W, [21, b, i]) for i, (H, W) in enumerate(shapes)])
    batches.append(batches[0])                       # replay an earlier batch again
    for b, frames in enumerate(batches):
        print(f"[graph replay] batch {b}: {[tuple(f.shape) for f in frames]}", flush=True)
        assert gb.fits([tuple(f.shape) for f in frames])
        outs = gb(frames)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device=DEV)
        junk.mul_(2.0).sum().item()
        for f, o in zip(frames, outs):
            want = api.complete(f)
            torch.cuda.synchronize()
            assert np.array_equal(bits(o), bits(want)), f"batch {b} frame {tuple(f.shape)}"
    # each pinned plan's first run without a frame under 3 rows or columns
    # captures its graph; later such runs replay it; batches with one run
    # eagerly with every launch step
    captured, want_replays = [False, False], 0
    for b, frames in enumerate(batches):
        if any(f.shape[0] < 3 or f.shape[1] < 3 for f in frames):
            continue
        if captured[b % 2]:
            want_replays += 1
        captured[b % 2] = True
    assert gb.replays == want_replays and want_replays >= 2
    m = batches[1][0].cpu().numpy()
    assert np.array_equal(bits(torch.from_numpy(oracle.complete_map(m))), bits(api.complete(batches[1][0])))


def test_graph_batch_rejects_oversized_batches():
    gb = batch.GraphBatch([(64, 128)] * 2, device=torch.device(DEV))
    assert not gb.fits([(64, 128)] * 3)
    assert not gb.fits([(65, 128)] * 2)
    assert gb.fits([(65, 128)])                         # one larger frame within the two-frame totals
    with pytest.raises(ValueError):
        gb.run([torch.zeros((64, 128), device=DEV)] * 3)


def test_graph_batch_uneven_workload_sample_equals_oracle():
    frames = [torch.from_numpy(f.sparse).to(DEV) for f in synth.config_frames(3, limit=5)]
    gb = batch.GraphBatch.for_batch(frames)
    for rep in range(3):
        outs = gb(frames)
        torch.cuda.synchronize()
        for i, (f, o) in enumerate(zip(frames, outs)):
            if rep == 0 and i < 2:
                want = oracle.complete_map(f.cpu().numpy())
                assert np.array_equal(bits(o), np.asarray(want, np.float32).view(np.uint32))
            assert np.array_equal(bits(o), bits(api.complete(f)))


def test_autotune_picks_a_valid_pair_and_results_do_not_change(tmp_path, monkeypatch):
    monkeypatch.setenv("IPB_TUNE_CACHE", str(tmp_path / "tune.json"))
    frames = [lidar(int(h), int(w), [22, i]) for i, (h, w) in enumerate([(256, 800), (300, 1100), (512, 2000)])]
    report = []
    p = autotune.tune(frames, reps=2, report=report)
    assert 1 <= p.tile_local <= ntiles(1) and 1 <= p.tile_global <= ntiles(2)
    assert any(r["us"] is not None for r in report)
    again = autotune.tune(frames, reps=2)              # from the cache
    assert (again.tile_local, again.tile_global) == (p.tile_local, p.tile_global)
    outs = api.complete_batch(frames, p)
    for f, o in zip(frames, outs):
        assert np.array_equal(bits(o), bits(api.complete(f)))


def test_autotune_for_batches_in_flight(tmp_path, monkeypatch):
    """tune(streams=2): the pairs are timed as batches in flight on two
    streams; the pick is a valid pair, cached apart from the one-stream
    pick, and results do not change."""
    monkeypatch.setenv("IPB_TUNE_CACHE", str(tmp_path / "tune.json"))
    frames = [lidar(int(h), int(w), [24, i]) for i, (h, w) in enumerate([(256, 800), (375, 1242), (300, 1100)])]
    report = []
    p = autotune.tune(frames, reps=2, report=report, streams=2)
    assert 1 <= p.tile_local <= ntiles(1) and 1 <= p.tile_global <= ntiles(2)
    pairs = [r for r in report if r["phase"] == "2 streams"]
    assert pairs and any(r["us"] is not None for r in pairs)
    assert f"{p.tile_local}/{p.tile_global}" in [r["tile"] for r in pairs]
    cache = json.load(open(tmp_path / "tune.json"))
    assert len(cache) == 1 and next(iter(cache)).endswith("|streams2")
    outs = api.complete_batch(frames, p)
    for f, o in zip(frames, outs):
        assert np.array_equal(bits(o), bits(api.complete(f)))


@pytest.mark.parametrize("executor", ["graph", "graph_only", "per_frame"])
def test_served_results_equal_alone(executor):
    rng = np.random.default_rng(23)
    shapes = [(352, 1216), (375, 1242), (200, 640), (96, 333)]
    p140 = api.Params(max_depth=140.0)
    frames, params = [], []
    for i in range(40):
        H, W = shapes[int(rng.integers(len(shapes)))]
        frames.append(lidar(H, W, [23, i], density=float(rng.uniform(0.02, 0.1))))
        params.append(p140 if i % 5 == 0 else None)
    if executor.startswith("graph"):
        # "graph": lone requests go straight to ipb_complete_ws; "graph_only": every batch replays a graph
        ex = serve.GraphExecutor(slots=3, max_batch=4, direct_single=executor == "graph")
    else:
        ex = serve.PerFrameExecutor()
    srv = serve.Server(ex, mem_budget=256 << 20, max_batch=4 if executor.startswith("graph") else 1)
    arrivals = np.cumsum(rng.exponential(1 / 4000.0, len(frames)))
    stats = serve.run_trace(srv, frames, arrivals, params)
    torch.cuda.synchronize()
    print(f"[serve {executor}] {stats}", flush=True)
    assert stats["completed"] == len(frames) and stats["rejected"] == 0
    by_id = {r.rid: r for r in srv.done}
    for i, f in enumerate(frames):
        alone = api.complete(f, params[i] or api.Params())
        torch.cuda.synchronize()
        assert np.array_equal(bits(by_id[i].out), bits(alone)), f"request {i}"
    if executor.startswith("graph"):
        assert ex.tiers == [1, 4]
        assert {len(eng.capacity) for eng in ex.engines.values()} <= {1, 4}


@pytest.mark.parametrize("executor", ["graph", "per_frame"])
def test_served_frames_produced_on_another_stream(executor):
    """Frames copied to the device on a producer stream (behind a long
    kernel there) and submitted right away, with no synchronisation: the
    server orders its launches after the producer's work, so every result
    equals the frame completed alone; outputs released by the client are
    reused only after the client's stream is done with them."""
    rng = np.random.default_rng(29)
    shapes = [(352, 1216), (200, 640), (96, 333)]
    host = []
    for i in range(24):
        H, W = shapes[i % len(shapes)]
        m = synth.lidar_frame(H, W, seed=[29, i], n_rows=min(64, H), density=float(rng.uniform(0.03, 0.08))).sparse
        host.append(torch.from_numpy(m).pin_memory())
    if executor == "graph":
        ex = serve.GraphExecutor(slots=3, max_batch=4)
    else:
        ex = serve.PerFrameExecutor()
    srv = serve.Server(ex, mem_budget=256 << 20, max_batch=4 if executor == "graph" else 1)
    producer = torch.cuda.Stream()
    junk = torch.ones(32 << 20, device=DEV)
    frames, reqs, copies = [], [], []
    print(f"[serve {executor}] frames from a producer stream", flush=True)
    with torch.cuda.stream(producer):
        for i, h in enumerate(host):
            junk.mul_(1.0)                               # keeps the producer stream busy ahead of the copy
            d = h.to(DEV, non_blocking=True)
            frames.append(d)
            reqs.append(srv.submit(d))
            srv.step()
            done = [r for r in srv.done if r.out is not None and r.status == "done"]
            for r in done:                               # the client reads an output on its stream, then releases it
                copies.append((r.rid, r.out.clone()))
                srv.release(r)
    srv.drain()
    torch.cuda.synchronize()
    for r in srv.done:
        if r.out is not None:
            copies.append((r.rid, r.out.clone()))
    torch.cuda.synchronize()
    assert len(copies) == len(host) and all(r.status in ("done", "released") for r in reqs)
    for rid, o in copies:
        alone = api.complete(frames[rid])
        torch.cuda.synchronize()
        assert np.array_equal(bits(o), bits(alone)), f"request {rid}"


def test_complete_on_a_stream_other_than_the_current_one():
    """api.complete / complete_batch on a non-current stream: buffers are
    allocated under that stream and inputs recorded on it, so work queued
    meanwhile on the current stream (allocating and freeing memory) cannot
    take them over."""
    f = lidar(375, 1242, [30, 0])
    g = [lidar(200, 640, [30, 1]), lidar(96, 333, [30, 2])]
    want = [bits(api.complete(x)) for x in [f] + g]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    junk = torch.ones(64 << 20, device=DEV)
    with torch.cuda.stream(s):
        junk.mul_(1.0)                                   # delays the calls below on s
    out = api.complete(f, stream=s)
    outs = api.complete_batch(g, stream=s)
    for _ in range(8):                                   # churn of the current stream's allocations
        t = torch.empty(4 * 375 * 1242 // 4 + 1024, device=DEV).fill_(-1.0)
        del t
    s.synchronize()
    assert np.array_equal(bits(out), want[0])
    for o, w in zip(outs, want[1:]):
        assert np.array_equal(bits(o), w)


def test_complete_batch_captured_into_a_graph():
    """ipb_complete_batch allocates nothing and waits for nothing, so it can
    be captured: replays of the captured call (with eager work and
    synchronisations between them) equal the eager call and each frame
    completed alone."""
    import ctypes
    shapes = [(375, 1242), (200, 640), (96, 333), (1, 7), (64, 64)]
    frames = [lidar(H, W, [32, i]) for i, (H, W) in enumerate(shapes)]
    # more descriptors than one upload chunk holds (the plan spans several launches)
    frames += [lidar(40, 90, [32, 10 + i]) for i in range(60)]
    outs = [torch.full_like(f, -1.0) for f in frames]
    p = api.Params().to_c()
    arr = api.frames_array(frames, outs)
    lib = L.lib()
    nb = int(lib.ipb_batch_workspace_bytes(arr, len(frames), ctypes.byref(p)))
    ws = api._workspace(nb, frames[0].device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        L.check(lib.ipb_complete_batch(arr, len(frames), ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nb,
                                       ctypes.c_void_p(s.cuda_stream)), "ipb_complete_batch")
    want = [bits(api.complete(f)) for f in frames]
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device=DEV)
        junk.mul_(2.0).sum().item()
        for i, (o, w) in enumerate(zip(outs, want)):
            assert np.array_equal(bits(o), w), f"replay {rep} frame {i} {tuple(frames[i].shape)}"


def test_quality_sweep_runs_every_design_step():
    from paper_1802_00036_amd import quality
    frames = [synth.lidar_frame(120, 300, seed=[24, i], n_rows=40, density=0.05) for i in range(2)]
    rows = quality.sweep(frames, quality.design_variants(api.Params()))
    assert len(rows) == 13
    for r in rows:
        assert np.isfinite(r["rmse_mm"]) and np.isfinite(r["mae_mm"]) and 0.0 <= r["coverage"] <= 1.0
    # the scored output is the library's: the default design equals the oracle
    f = frames[0]
    got = api.complete(torch.from_numpy(f.sparse).to(DEV)).cpu().numpy()
    want = oracle.complete_map(f.sparse)
    assert np.array_equal(got.view(np.uint32), np.asarray(want, np.float32).view(np.uint32))
    assert np.isclose(rows[-1]["rmse_mm"], quality.pooled(
        [api.complete(torch.from_numpy(fr.sparse).to(DEV)).cpu().numpy() for fr in frames],
        [fr.dense_gt for fr in frames])["rmse_mm"], rtol=1e-3)


def _planned_steps(frames, outs, p, steps=range(5)):
    """The bench's launch configuration: one plan for the whole batch, then
    ipb_complete_planned one launch step at a time (steps 0-4: no frame has
    under 3 rows or columns); steps may also be [-1] or [-2]."""
    import ctypes
    from paper_1802_00036_amd import _lib as L
    lib = L.lib()
    cp = p.to_c()
    arr = api.frames_array(frames, outs)
    nb = int(lib.ipb_batch_workspace_bytes(arr, len(frames), ctypes.byref(cp)))
    ws = api._workspace(nb, frames[0].device)
    pb = int(lib.ipb_batch_plan_bytes(len(frames)))
    ph = ctypes.create_string_buffer(pb)
    L.check(lib.ipb_batch_plan(arr, len(frames), ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), nb, ph, pb),
            "ipb_batch_plan")
    n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
    lib.ipb_plan_totals(ph, ctypes.byref(n), ctypes.byref(lt), ctypes.byref(gt), ctypes.byref(cols))
    pd = torch.frombuffer(bytearray(ph.raw), dtype=torch.uint8).to(frames[0].device)
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for step in steps:
        L.check(lib.ipb_complete_planned(ctypes.c_void_p(pd.data_ptr()), ctypes.byref(cp), step, lt.value, gt.value,
                                         cols.value, sh), "ipb_complete_planned")
    torch.cuda.synchronize()
    del ws, pd


@pytest.mark.parametrize("whole", [-1, -2])
def test_planned_whole_launch(whole):
    """ipb_complete_planned with every step at once (-1), and without the
    step of frames under 3 rows or columns (-2) on frames that have none
    (sizes down to 3 rows and 3 columns): each frame bitwise equal to the
    frame completed alone."""
    shapes = [(3, 200), (200, 3), (3, 3), (64, 64), (97, 300), (375, 1242)]
    rng = np.random.default_rng(11)
    frames = []
    for H, W in shapes:
        d = np.where(rng.random((H, W)) < 0.06, rng.uniform(1.0, 80.0, (H, W)), 0.0).astype(np.float32)
        frames.append(torch.from_numpy(d).to(DEV))
    outs = [torch.empty_like(t) for t in frames]
    p = api.Params()
    print(f"[planned whole {whole}] shapes {shapes}", flush=True)
    _planned_steps(frames, outs, p, steps=[whole])
    for i, (t, o) in enumerate(zip(frames, outs)):
        assert np.array_equal(bits(o), bits(api.complete(t, p))), f"frame {i} {shapes[i]}: batch != alone"


def test_graph_pipeline_matches_alone():
    """GraphPipeline: batches of uneven frames on three engines in turn
    (each engine's first two batches eager, one per pinned plan, later ones
    graph replays), several batches in flight at once: every output bitwise
    equal to the frame completed alone."""
    rng = np.random.default_rng(41)
    cap = [(300, 900), (200, 640), (375, 1242)]
    pipe = batch.GraphPipeline(cap, engines=3)
    jobs = []
    for b in range(9):
        shapes = [(int(rng.integers(100, 301)), int(rng.integers(300, 901))), (200, 640), (375, 1242)]
        frames = [lidar(H, W, [41, b, i]) for i, (H, W) in enumerate(shapes)]
        outs = [torch.empty_like(f) for f in frames]
        jobs.append((frames, outs))
    torch.cuda.synchronize()
    print("[graph pipeline] 9 batches on 3 engines", flush=True)
    events = [pipe.run(frames, outs) for frames, outs in jobs]
    for e in events:
        e.synchronize()
    assert sum(e.replays for e in pipe.engines) == 3       # the third batch of each engine is a replay
    for b, (frames, outs) in enumerate(jobs):
        for i, (f, o) in enumerate(zip(frames, outs)):
            assert np.array_equal(bits(o), bits(api.complete(f))), f"batch {b} frame {i}"


def test_shipped_tuning_entry_is_found(tmp_path, monkeypatch):
    """On MI355X the shipped table answers tune() for the 64 x 375x1242
    benchmark batch at three streams: no candidate is timed."""
    monkeypatch.setenv("IPB_TUNE_CACHE", str(tmp_path / "empty.json"))
    frames = [torch.from_numpy(f.sparse).to(DEV) for f in synth.config_frames(2)]
    table = json.load(open(autotune.SHIPPED_TABLE))
    key = "|".join((autotune.device_signature(frames[0].device), autotune.params_signature(api.Params()),
                    autotune.batch_signature([tuple(f.shape) for f in frames]), "streams3"))
    if key not in table:
        pytest.skip(f"not the device the table was measured on ({autotune.device_signature(frames[0].device)})")
    report = []
    p = autotune.tune(frames, report=report, streams=3)
    assert report == []
    assert (p.tile_local, p.tile_global) == (table[key]["tile_local"], table[key]["tile_global"])


def test_queue_streams_have_queues_of_their_own():
    """ipb_stream_create: three streams with distinct handles, made once per
    device (a second request returns the same ones), whose work runs side by
    side: three equal spin kernels, one per stream, end in well under the
    time they take one after the other."""
    qs = api.queue_streams(3)
    assert len({s.cuda_stream for s in qs}) == 3
    assert [s.cuda_stream for s in api.queue_streams(2)] == [s.cuda_stream for s in qs[:2]]

    def spin(streams, cycles):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(qs[0])
        for s in streams[1:]:
            s.wait_event(a)
        for s in streams:
            with torch.cuda.stream(s):
                torch.cuda._sleep(cycles)
        for s in streams[1:]:
            e = torch.cuda.Event()
            e.record(s)
            qs[0].wait_event(e)
        b.record(qs[0])
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    spin(qs[:1], 1 << 20)
    cycles = max(1 << 20, int((1 << 20) * 10.0 / spin(qs[:1], 1 << 20)))    # about 10 ms
    one = spin(qs[:1], cycles)
    three = spin(qs, cycles)
    print(f"[queue streams] one spin {one:.2f} ms, three side by side {three:.2f} ms", flush=True)
    assert three < 2.0 * one


def test_queue_streams_fall_back_to_pool_streams(monkeypatch):
    """A runtime that refuses a compute-unit-masked stream: queue_streams
    warns and hands out torch's pool streams, on which a batch still
    completes bitwise as the frame alone."""
    lib = L.lib()
    calls = []

    def refuse(ptr):
        calls.append(ptr)
        return L.IPB_ERR_HIP

    monkeypatch.setattr(api, "_QUEUE_STREAMS", {})
    monkeypatch.setattr(lib, "ipb_stream_create", refuse)
    with pytest.warns(RuntimeWarning, match="pool streams"):
        qs = api.queue_streams(2)
    assert len(calls) == 2 and all(not isinstance(s, torch.cuda.ExternalStream) for s in qs)
    f = lidar(200, 640, [61])
    torch.cuda.synchronize()
    with torch.cuda.stream(qs[1]):
        out = api.complete_batch([f])[0]
    qs[1].synchronize()
    assert np.array_equal(bits(out), bits(api.complete(f)))


@pytest.mark.parametrize("shape,n,tiles", [((375, 1242), 5, (10, 5)), ((3, 3), 4, (0, 0)), ((130, 301), 7, (5, 6)),
                                            ((64, 120), 9, (10, 7)), ((1024, 250), 3, (6, 7)), ((17, 4096), 2, (7, 8)),
                                            ((200, 640), 6, (8, 9))])
def test_batch_of_one_shape_equals_alone(shape, n, tiles):
    """A batch whose frames share one shape takes phase 2's tiles bottom tile
    row first over all frames (from the plan's shared tiling): every output
    bitwise equal to the frame completed alone, for frames of one tile and
    of many, odd widths, the 3 x 3 minimum and each phase-2 tile height of
    the default chain (64, 32, 128, 16 and 8 rows)."""
    H, W = shape
    frames = [lidar(H, W, [53, H, i]) for i in range(n)]
    p = dataclasses.replace(api.Params(), tile_local=tiles[0], tile_global=tiles[1])
    print(f"[one shape] {n} x {H}x{W}, tiles {tiles}", flush=True)
    outs = api.complete_batch(frames, p)
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(frames, outs)):
        assert np.array_equal(bits(o), bits(api.complete(f))), f"frame {i}"


@pytest.mark.parametrize("kind", ["pool", "queue"])
def test_batches_in_flight_on_streams(kind):
    """Three batches in flight on three streams (torch's pool streams, or
    streams with hardware queues of their own), each with its own outputs,
    workspace and plan, the inputs shared and only read, several rounds as
    the bench's timed pass runs them: every output bitwise equal to the
    frame completed alone."""
    import ctypes
    from paper_1802_00036_amd import _lib as L
    lib = L.lib()
    rng = np.random.default_rng(31)
    shapes = [(375, 1242), (200, 640), (96, 333), (375, 1242)]
    frames = [lidar(H, W, [31, i], density=float(rng.uniform(0.03, 0.08))) for i, (H, W) in enumerate(shapes)]
    p = dataclasses.replace(api.Params(), tile_local=6, tile_global=6)
    cp = p.to_c()
    lanes = []
    for k in range(3):
        outs = [torch.empty_like(f) for f in frames]
        arr = api.frames_array(frames, outs)
        nb = int(lib.ipb_batch_workspace_bytes(arr, len(frames), ctypes.byref(cp)))
        ws = api._workspace(nb, frames[0].device)
        pb = int(lib.ipb_batch_plan_bytes(len(frames)))
        ph = ctypes.create_string_buffer(pb)
        L.check(lib.ipb_batch_plan(arr, len(frames), ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), nb, ph, pb),
                "ipb_batch_plan")
        n, lt, gt, cols = (ctypes.c_int() for _ in range(4))
        lib.ipb_plan_totals(ph, ctypes.byref(n), ctypes.byref(lt), ctypes.byref(gt), ctypes.byref(cols))
        pd = torch.frombuffer(bytearray(ph.raw), dtype=torch.uint8).to(frames[0].device)
        st = torch.cuda.Stream() if kind == "pool" else api.queue_streams(3)[k]
        lanes.append((st, outs, ws, pd, lt.value, gt.value, cols.value))
    torch.cuda.synchronize()
    print(f"[in flight] 3 {kind} streams x 6 rounds", flush=True)
    for _ in range(6):
        for s, outs, ws, pd, lt, gt, cols in lanes:
            L.check(lib.ipb_complete_planned(ctypes.c_void_p(pd.data_ptr()), ctypes.byref(cp), -2, lt, gt, cols,
                                             ctypes.c_void_p(s.cuda_stream)), "ipb_complete_planned")
    torch.cuda.synchronize()
    for k, (_, outs, *_rest) in enumerate(lanes):
        for i, (f, o) in enumerate(zip(frames, outs)):
            assert np.array_equal(bits(o), bits(api.complete(f))), f"stream {k} frame {i} {shapes[i]}"


@pytest.mark.parametrize("cfg", [2, 4])
def test_bench_configuration_full_batch(cfg):
    """The whole batch the bench times (64 x 375x1242; 16 x 1024x4096) with
    the tiles the bench takes for it (the shipped tuning table's entry for
    three streams, as on a box without a user cache), in the bench's launch
    configuration: every frame bitwise equal to the frame completed alone,
    and frames spread over the batch equal to the oracle."""
    from paper_1802_00036_amd import autotune
    p = api.Params(max_depth=140.0) if cfg == 4 else api.Params()
    fr = synth.config_frames(cfg)
    frames = [torch.from_numpy(f.sparse).to(DEV) for f in fr]
    tuned = autotune.lookup(frames, p, streams=3, user_cache=False)
    assert tuned is not None, f"the shipped tuning table has no entry for c{cfg}"
    p = tuned
    outs = [torch.empty_like(t) for t in frames]
    print(f"[bench config c{cfg}] {len(frames)} frames, tiles {p.tile_local}/{p.tile_global}", flush=True)
    _planned_steps(frames, outs, p)
    alone = dataclasses.replace(p, tile_local=0, tile_global=0)   # the library's tiles for one frame
    for i, (t, o) in enumerate(zip(frames, outs)):
        assert np.array_equal(bits(o), bits(api.complete(t, alone))), f"c{cfg} frame {i}: batch != alone"
    sample = [0, len(fr) // 2, len(fr) - 1] if cfg == 4 else [0, 9, 21, 33, 47, 63]
    for i in sample:
        want = oracle.complete_map(fr[i].sparse, oracle.Params(max_depth=p.max_depth))
        got = np.ascontiguousarray(outs[i].cpu().numpy())
        assert np.array_equal(got.view(np.uint32), np.ascontiguousarray(want, np.float32).view(np.uint32)), \
            f"c{cfg} frame {i} differs from the oracle"
