"""Host-side tests of the serving scheduler and the batch helpers (no GPU):
admission by memory budget, size buckets, continuous batching over slots,
rejection, statistics, and the autotuner's cache."""
import collections
import dataclasses
import json

import numpy as np
import pytest

from paper_1802_00036_amd import serve


class FakeClock:
    def __init__(self, step=1e-4):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor(serve.Executor):
    """Batches finish after `polls` readiness checks; outputs are the
    frames themselves.  Records how many batches were running at each launch."""

    def __init__(self, slots=2, polls=3, in_order=False):
        self.slots = slots
        self.polls = polls
        self.in_order = in_order
        self.live = 0
        self.launches = []          # (slot, bucket, rids, batches running after this launch)

    def launch(self, slot, bucket, reqs):
        self.live += 1
        self.launches.append((slot, bucket, [r.rid for r in reqs], self.live))
        return {"left": self.polls, "outs": [r.frame for r in reqs], "slot": slot}

    def ready(self, h):
        h["left"] -= 1
        if h["left"] <= 0 and not h.get("counted"):
            h["counted"] = True
            self.live -= 1
        return h["left"] <= 0

    def outputs(self, h):
        return h["outs"]

    def recycle(self, outs, by_client=True):
        self.recycled = getattr(self, "recycled", 0) + len(outs)


class Frame:
    def __init__(self, H, W, tag):
        self.shape = (H, W)
        self.tag = tag


def make_server(slots=2, polls=3, budget=10**9, max_batch=4, max_queue=1000, in_order=False, keep=True):
    ex = FakeExecutor(slots, polls, in_order)
    return serve.Server(ex, mem_budget=budget, max_batch=max_batch, max_queue=max_queue, clock=FakeClock(),
                        keep_outputs=keep), ex


def test_every_request_completes_once_with_its_own_output():
    srv, ex = make_server()
    shapes = [(352, 1216), (375, 1242), (512, 2048), (1024, 4096)]
    rng = np.random.default_rng(0)
    reqs = [srv.submit(Frame(*shapes[int(rng.integers(4))], i)) for i in range(57)]
    srv.drain()
    assert all(r.status == "done" for r in reqs)
    assert sorted(r.rid for r in srv.done) == list(range(57))
    assert all(r.out.tag == r.rid for r in reqs)
    assert srv.in_use == sum(r.nbytes for r in reqs)      # kept outputs stay counted until released
    for r in reqs:
        srv.release(r)
    assert srv.in_use == 0


def test_batches_are_bucketed_fifo_and_bounded():
    srv, ex = make_server(max_batch=3)
    shapes = [(352, 1216), (375, 1242), (300, 1200)]     # buckets: 384x1216, 384x1280, 320x1216
    for i in range(30):
        srv.submit(Frame(*shapes[i % 3], i))
    srv.drain()
    by_rid = {r.rid: r for r in srv.done}
    for slot, bucket, rids, _ in ex.launches:
        assert 1 <= len(rids) <= 3
        assert len({by_rid[i].bucket for i in rids}) == 1
        assert rids == sorted(rids)
    # within a bucket, launches follow arrival order
    seen = collections.defaultdict(list)
    for _, bucket, rids, _ in ex.launches:
        seen[bucket].extend(rids)
    for rids in seen.values():
        assert rids == sorted(rids)


def test_default_bucket_rounds_up_to_64():
    assert serve.default_bucket((375, 1242)) == (384, 1280)
    assert serve.default_bucket((64, 64)) == (64, 64)
    assert serve.default_bucket((1, 1)) == (64, 64)


def test_continuous_batching_overlaps_slots():
    srv, ex = make_server(slots=3, polls=50, max_batch=2)
    for i in range(4):
        srv.submit(Frame(64, 64, i))
    srv.step()                                  # two batches of two start at once
    for i in range(4, 6):
        srv.submit(Frame(64, 64, i))
    srv.step()                                  # arrivals start on the third slot while the others run
    assert max(l[3] for l in ex.launches) == 3
    srv.drain()
    assert len(srv.done) == 6


def test_memory_budget_bounds_admission():
    frame_bytes = 4 * 100 * 100
    srv, ex = make_server(slots=4, polls=5, budget=3 * frame_bytes, max_batch=8, keep=False)
    for i in range(10):
        srv.submit(Frame(100, 100, i))
    srv.step()
    assert srv.in_use == 3 * frame_bytes
    assert len(srv.waiting) == 7
    srv.drain()
    assert srv.peak_in_use <= 3 * frame_bytes
    assert len(srv.done) == 10 and not srv.rejected
    assert ex.recycled == 10 and srv.in_use == 0


def test_kept_outputs_hold_the_budget_until_released():
    frame_bytes = 4 * 100 * 100
    srv, ex = make_server(slots=2, polls=2, budget=2 * frame_bytes, max_batch=8)
    reqs = [srv.submit(Frame(100, 100, i)) for i in range(4)]
    with pytest.raises(RuntimeError):
        srv.drain()                       # two outputs held, the next cannot be admitted
    assert [r.status for r in reqs] == ["done", "done", "queued", "queued"]
    srv.release(reqs[0])
    srv.release(reqs[1])
    assert srv.in_use == 0 and reqs[0].out is None and reqs[0].status == "released"
    srv.release(reqs[0])                  # a second release changes nothing
    assert srv.in_use == 0
    srv.drain()
    assert [r.status for r in reqs[2:]] == ["done", "done"]
    assert srv.in_use == 2 * frame_bytes


def test_rejections():
    srv, _ = make_server(budget=4 * 64 * 64, max_queue=2)
    big = srv.submit(Frame(128, 128, 0))                    # larger than the whole budget
    assert big.status == "rejected"
    a, b, c = (srv.submit(Frame(8, 8, i)) for i in range(3))   # queue holds two
    assert (a.status, b.status, c.status) == ("queued", "queued", "rejected")
    srv.drain()
    assert srv.stats()["rejected"] == 2
    assert srv.stats()["completed"] == 2


def test_in_order_executor_polls_only_the_oldest():
    srv, ex = make_server(slots=8, polls=2, max_batch=1, in_order=True)
    for i in range(5):
        srv.submit(Frame(16, 16, i))
    srv.drain()
    done_order = [r.rid for r in srv.done]
    assert done_order == sorted(done_order)


def test_stats_and_run_trace():
    srv, _ = make_server(slots=2, polls=2, max_batch=4, keep=False)
    frames = [Frame(64, 128, i) for i in range(40)]
    arrivals = np.cumsum(np.full(40, 1e-3))
    st = serve.run_trace(srv, frames, arrivals, warmup=0.0055)
    assert st["completed"] == int(np.sum(arrivals >= 0.0055)) == 35
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["wait_p99_ms"] >= 0 and 0 < st["service_p50_ms"] <= st["service_p99_ms"]
    assert st["frames_per_batch"] >= 1
    assert st["throughput_fps"] > 0
    lat = [r.latency for r in srv.done]
    assert min(lat) > 0


def test_params_split_buckets():
    @dataclasses.dataclass
    class P:
        max_depth: float = 100.0

    srv, ex = make_server(max_batch=8)
    for i in range(6):
        srv.submit(Frame(64, 64, i), params=P(100.0 if i % 2 else 140.0))
    srv.drain()
    for _, bucket, rids, _ in ex.launches:
        assert len({i % 2 for i in rids}) == 1


# ---------------------------------------------------------------- autotune --

def test_autotune_signatures_and_cache(tmp_path, monkeypatch):
    from paper_1802_00036_amd import autotune
    from paper_1802_00036_amd.api import Params
    a = autotune.batch_signature([(375, 1242)] * 64)
    b = autotune.batch_signature([(376, 1240)] * 64)
    c = autotune.batch_signature([(375, 1242)] * 8)
    assert a == b and a != c
    assert autotune.params_signature(Params(tile_local=5)) == autotune.params_signature(Params(tile_global=3))
    assert autotune.params_signature(Params()) != autotune.params_signature(Params(max_depth=140.0))
    path = tmp_path / "tune.json"
    monkeypatch.setenv("IPB_TUNE_CACHE", str(path))
    assert autotune.cache_path() == str(path)
    autotune._store_cache(str(path), "k1", {"tile_local": 5, "tile_global": 6})
    autotune._store_cache(str(path), "k2", {"tile_local": 7, "tile_global": 5})
    data = json.loads(path.read_text())
    assert data["k1"]["tile_local"] == 5 and data["k2"]["tile_global"] == 5
    path.write_text("not json")
    assert autotune._load_cache(str(path)) == {}


def test_shapes_workspace_bytes_matches_layout():
    from paper_1802_00036_amd import batch
    from paper_1802_00036_amd.api import Params
    one = batch.shapes_workspace_bytes([(375, 1242)])
    two = batch.shapes_workspace_bytes([(375, 1242), (375, 1242)])
    assert two > one > 2 * 4 * 375 * 1242
    assert two - one >= 2 * 4 * 375 * 1242
    # larger frames never need less workspace
    assert batch.shapes_workspace_bytes([(400, 1300)]) >= one
    lt, gt, cols = batch._tile_counts(Params().to_c(), [(375, 1242), (64, 64)])
    assert cols == 1306 and lt > 0 and gt > 0


@pytest.mark.parametrize("shapes", [[(352, 1216)], [(375, 1242)], [(512, 2048)], [(1024, 4096)],
                                    [(375, 1242)] * 4, [(375, 1242)] * 8, [(375, 1242)] * 16,
                                    [(1024, 4096)] * 2, [(375, 1242)] * 64])
@pytest.mark.parametrize("chain", ["default", "median3", "cross"])
def test_graph_batch_tile_rule_matches_the_library(shapes, chain):
    """batch.auto_tiles picks the tiles the library picks for calls that see
    the frames: the batch workspace for the automatic ids (which covers the
    library's pick and the default tiles) equals the larger of the two
    layouts for the explicit ids batch.auto_tiles returns."""
    from paper_1802_00036_amd import api, batch
    from paper_1802_00036_amd.api import Params
    p = {"default": Params(), "median3": Params(median_size=3),
         "cross": Params(dilate_shape=api.SE_CROSS)}[chain]
    picked = batch.auto_tiles(p, shapes)
    lib_bytes = batch.shapes_workspace_bytes(shapes, p)
    explicit = batch.shapes_workspace_bytes(shapes, picked)
    # the library's default ids: the streaming kernels where the chain has them
    tl = 5 if batch._placeholder_bytes(shapes, dataclasses.replace(p, tile_local=5, tile_global=1)) else 1
    tg = 6 if batch._placeholder_bytes(shapes, dataclasses.replace(p, tile_local=tl, tile_global=6)) else 1
    default = batch.shapes_workspace_bytes(shapes, dataclasses.replace(p, tile_local=tl, tile_global=tg))
    assert lib_bytes == max(explicit, default)
    if chain == "median3":
        assert picked.tile_global == 0                  # 16- and 8-row phase-2 tiles: 5x5 median chains only


# ------------------------------------------------------- failure handling --

class FailingExecutor(FakeExecutor):
    """Launches whose requests include a rid in `bad_launch` raise at
    launch; batches holding a rid in `bad_done` raise when polled.  A set
    entry "alone" fails only when the request runs alone, "batch" only in a
    batch of several, "always" both times."""

    def __init__(self, bad_launch=None, bad_done=None, **kw):
        super().__init__(**kw)
        self.bad_launch = bad_launch or {}
        self.bad_done = bad_done or {}
        self.attempts = collections.Counter()

    @staticmethod
    def _hit(table, reqs):
        for r in reqs:
            mode = table.get(r.rid)
            if mode == "always" or (mode == "alone" and len(reqs) == 1) or (mode == "batch" and len(reqs) > 1):
                return True
        return False

    def launch(self, slot, bucket, reqs):
        for r in reqs:
            self.attempts[r.rid] += 1
        if self._hit(self.bad_launch, reqs):
            raise RuntimeError("launch failed")
        h = super().launch(slot, bucket, reqs)
        h["fail"] = self._hit(self.bad_done, reqs)
        return h

    def ready(self, h):
        ok = super().ready(h)
        if ok and h["fail"]:
            raise RuntimeError("device fault reported at completion")
        return ok


def _failing_server(**kw):
    ex = FailingExecutor(slots=2, polls=2, **kw)
    return serve.Server(ex, mem_budget=10**9, max_batch=4, clock=FakeClock()), ex


def test_failed_batch_is_retried_alone_once():
    """A batch whose launch raises (request 2 poisons any batch it is in):
    every request of it is retried alone; those that then succeed complete,
    and no request is launched more than twice."""
    srv, ex = _failing_server(bad_launch={2: "batch"})
    reqs = [srv.submit(Frame(64, 64, i)) for i in range(4)]
    srv.drain()
    assert all(r.status == "done" for r in reqs)
    assert srv.failed_batches == 1
    assert all(ex.attempts[r.rid] == 2 for r in reqs)
    assert all(r.solo for r in reqs)
    assert srv.in_use == sum(r.nbytes for r in reqs)


def test_request_failing_alone_is_marked_failed():
    """Request 1 fails every time: after its batch fails and its solo retry
    fails, it is marked failed with the error; its memory leaves the budget
    and the others complete."""
    srv, ex = _failing_server(bad_launch={1: "always"})
    reqs = [srv.submit(Frame(64, 64, i)) for i in range(3)]
    srv.drain()
    assert [r.status for r in reqs] == ["done", "failed", "done"]
    assert "launch failed" in reqs[1].error
    assert ex.attempts[1] == 2
    assert srv.failed == [reqs[1]]
    assert srv.in_use == reqs[0].nbytes + reqs[2].nbytes
    assert srv.stats()["failed"] == 1


def test_failure_reported_at_completion_is_retried():
    """The device work of a batch fails (the end-of-batch query raises): the
    slot is freed, the batch's requests are retried alone, a lone request
    failing on its own is marked failed."""
    srv, ex = _failing_server(bad_done={0: "batch", 3: "always"})
    reqs = [srv.submit(Frame(64, 64, i)) for i in range(4)]
    srv.drain()
    assert [r.status for r in reqs] == ["done", "done", "done", "failed"]
    assert "device fault" in reqs[3].error
    assert sorted(srv.free_slots) == [0, 1]
    assert srv.idle()


def test_lone_request_failing_gets_one_retry():
    srv, ex = _failing_server(bad_launch={0: "always"})
    r = srv.submit(Frame(64, 64, 0))
    srv.drain()
    assert r.status == "failed" and ex.attempts[0] == 2


def test_cancel_in_every_state():
    srv, ex = make_server(slots=1, polls=5, max_batch=1, budget=3 * 4 * 64 * 64)
    reqs = [srv.submit(Frame(64, 64, i)) for i in range(6)]
    srv.step()                      # r0 runs, r1 and r2 are admitted, r3.. wait for memory
    assert [r.status for r in reqs[:4]] == ["running", "admitted", "admitted", "queued"]
    assert srv.cancel(reqs[3]) and reqs[3].status == "cancelled"       # waiting
    assert srv.cancel(reqs[1]) and reqs[1].status == "cancelled"       # admitted: its bytes leave
    assert srv.in_use == 2 * 4 * 64 * 64
    assert srv.cancel(reqs[0]) and reqs[0].status == "running"         # running: marked only
    srv.drain()
    assert reqs[0].status == "cancelled" and reqs[0].out is None
    assert [r.status for r in reqs[2:]] == ["done", "cancelled", "done", "done"]
    assert not srv.cancel(reqs[2])                                     # already finished
    assert srv.in_use == sum(r.nbytes for r in (reqs[2], reqs[4], reqs[5]))
    assert ex.recycled == 1                                            # r0's buffer went back
    assert {r.rid for r in srv.done} == {2, 4, 5}


def test_requests_time_out_before_launch():
    """With one slot held by a long batch, requests still waiting or admitted
    past their deadline time out (their bytes leave the budget); a running
    batch is never timed out; a request with its own longer timeout stays."""
    clock = FakeClock(step=1e-3)
    ex = FakeExecutor(slots=1, polls=40)
    srv = serve.Server(ex, mem_budget=10**9, max_batch=1, clock=clock, timeout=0.01)
    first = srv.submit(Frame(64, 64, 0))
    srv.step()
    late = [srv.submit(Frame(64, 64, i)) for i in range(1, 4)]
    patient = srv.submit(Frame(64, 64, 9), timeout=10.0)
    srv.step()                        # admitted, waiting for the slot
    for _ in range(30):
        srv.step()
    assert first.status in ("running", "done")
    assert all(r.status == "timeout" for r in late)
    srv.drain()
    assert first.status == "done" and patient.status == "done"
    assert srv.in_use == first.nbytes + patient.nbytes
    assert srv.stats()["timed_out"] == 3


class ResidentExecutor(FakeExecutor):
    """Holds `held` bytes of resident memory that trim() can drop."""

    def __init__(self, held, **kw):
        super().__init__(**kw)
        self.held = held
        self.trims = []

    def resident_bytes(self):
        return self.held

    def trim(self, target):
        self.trims.append(target)
        self.held = min(self.held, target)


def test_admission_counts_resident_memory():
    fb = 4 * 64 * 64
    ex = ResidentExecutor(held=3 * fb, slots=1, polls=3)
    srv = serve.Server(ex, mem_budget=5 * fb, max_batch=8, clock=FakeClock())
    reqs = [srv.submit(Frame(64, 64, i)) for i in range(4)]
    srv.step()
    # 3 frames' worth is resident: only two outputs fit beside it
    assert sum(r.status in ("admitted", "running") for r in reqs) == 2
    srv.drain()
    assert all(r.status == "done" for r in reqs)
    # the last two could only be admitted after trim() dropped idle memory
    # (outputs of the first two are kept, so 2 frames + 2 frames leave 1)
    assert ex.trims and ex.held <= fb
