"""The tuning table that ships with the package: well formed, every entry a
pair of tile ids the library knows, and keyed the way `autotune.tune` looks
entries up (device | parameters | batch signature | stream count)."""
import json

from paper_1802_00036_amd import _lib as L
from paper_1802_00036_amd import autotune, synth
from paper_1802_00036_amd.api import Params


def test_shipped_table_entries():
    table = json.load(open(autotune.SHIPPED_TABLE))
    assert table
    lib = L.lib()
    n_local, n_global = int(lib.ipb_tile_count(1)), int(lib.ipb_tile_count(2))
    for key, e in table.items():
        parts = key.split("|")
        assert len(parts) == 4 and parts[3] == f"streams{e['streams']}"
        assert "gfx950" in parts[0]
        assert 1 <= e["tile_local"] <= n_local and 1 <= e["tile_global"] <= n_global
        assert e["us_per_batch"] > 0


def test_shipped_table_covers_the_benchmark_batches():
    """The keys' parameter and batch parts are those tune() computes for the
    benchmark batches (workloads 2, 3, 4 of the generator) at three streams."""
    table = json.load(open(autotune.SHIPPED_TABLE))
    tails = {"|".join(k.split("|")[1:]) for k in table}
    for cfg in (2, 3, 4):
        shapes = [f.sparse.shape for f in synth.config_frames(cfg)]
        p = Params(max_depth=140.0) if cfg == 4 else Params()
        tail = "|".join((autotune.params_signature(p), autotune.batch_signature(shapes), "streams3"))
        assert tail in tails, f"no shipped entry for workload {cfg}"
