"""The path queue, camera connections and launch timing on the GPU: small and
ragged path counts (empty queue shards), a box scene with an escape sensor
(no camera work at all), and the library's launch timing."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from replay import compare_records, oracle_replay
from stats import check_z, escape_z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 129, 1000])
def test_small_path_counts_take_every_id_once(n):
    """Counts below, at and above the number of queue shards: every path id of
    [begin, begin + n) is walked exactly once and replays against the oracle."""
    import torch
    import paper_1706_03024_amd as fpt
    scene = workloads.cornell_scene(16, 16)
    run = workloads.make_run(n, seed=21, path_begin=777, total_paths=4096)
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    sc.render(run, tallies=t)
    rec, _ = sc.records(run)
    torch.cuda.synchronize()
    tal = fpt.tallies_dict(t)
    sc.close()
    assert tal["paths"] == n
    assert sum(tal["exit_" + e] for e in oracle.EXIT_NAMES) == n
    assert (rec["n_vertices"] >= 1).all()  # every record slot was written
    compare_records(rec, oracle_replay(scene, run))


def test_box_with_escape_sensor_makes_no_connections():
    """A box scene read by escape tallies evaluates no camera connection (the
    connection tallies stay 0) and its escape film agrees with the oracle."""
    scene = workloads.cornell_scene(8, 8)
    scene["sensor"] = {"kind": "escape"}
    import torch
    import paper_1706_03024_amd as fpt
    n_g, n_o = 1 << 20, 1 << 17
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    film = sc.render(workloads.make_run(n_g, seed=31), tallies=t)
    torch.cuda.synchronize()
    g = film.cpu().numpy().astype(np.float64)
    tal = fpt.tallies_dict(t)
    sc.close()
    assert tal["splat_hit"] == tal["splat_miss"] == tal["splat_rr_kill"] == 0
    o = oracle.render(scene, workloads.make_run(n_o, seed=32))
    assert o["tallies"][oracle.TALLY_NAMES.index("splat_miss")] == 0
    check_z(escape_z(g[0], n_g, o["film"][0], n_o), "box + escape sensor: GPU vs oracle")


@pytest.mark.parametrize("name", ["cornell", "slab"])
def test_launch_timing(name):
    """fpt_scene_timing returns the number of timed renders and positive mean
    launch durations; a pinhole render has a deferred-connection launch."""
    import torch
    import paper_1706_03024_amd as fpt
    scene, run = {"cornell": workloads.cornell_config, "slab": workloads.slab_config}[name]()
    sc = fpt.Scene(scene)
    film = sc.new_film()
    sc.set_timing(True)
    for _ in range(3):
        sc.render(run, film=film)
    n, t_ms, d_ms = sc.timing()
    assert n == 3 and t_ms > 0.0 and d_ms >= 0.0
    if name == "cornell":
        assert d_ms > 0.0
    assert sc.timing()[0] == 0  # the record was cleared
    sc.set_timing(False)
    sc.render(run, film=film)
    torch.cuda.synchronize()
    assert sc.timing()[0] == 0
    sc.close()


def test_path_count_limits():
    """Path ids are 32-bit: a call of 2^32 paths is refused (FPT_E_RANGE, no
    launch) while the last ids of a 2^32-path job render, each once, every
    escape weighing 1/2^32 (the job's total)."""
    import torch
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import _abi
    scene, run = workloads.slab_config()
    sc = fpt.Scene(scene)
    big = dict(run, path_begin=0, path_count=1 << 32, total_paths=1 << 32)
    with pytest.raises(fpt.FptError) as e:
        sc.render(big)
    assert e.value.status == _abi.E_RANGE
    tail = dict(run, path_begin=(1 << 32) - 100, path_count=100, total_paths=1 << 32)
    t = fpt.new_tallies()
    film = sc.render(tail, tallies=t)
    rec, _ = sc.records(tail)
    torch.cuda.synchronize()
    sc.close()
    td = fpt.tallies_dict(t)
    assert td["paths"] == 100
    escaped = td["exit_esc_r"] + td["exit_esc_t"]
    assert escaped > 50 and abs(float(film.double().sum()) * (1 << 32) - escaped) <= 1e-3
    compare_records(rec, oracle_replay(scene, tail))


def test_autotune_cache_owned_by_the_library(tmp_path):
    """fpt_autotune reads and writes the JSON cache itself: a cached entry is
    returned without measuring, an uncached workload with CACHED_ONLY gives
    the library defaults, a measured one is written back under the device's
    key, and a malformed cache is an error."""
    import json
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import autotune
    scene, run = workloads.slab_config()
    run = dict(run, path_count=1 << 14, total_paths=1 << 14)
    key = "probe@" + autotune.device_tag()
    path = tmp_path / "cache.json"
    entry = {"block_min_vertices": 3, "block_segments": 2, "block_threads": 192,
             "blocks_per_cu": 1, "chunk_paths": 0, "ms": 1.25, "refill_lanes": 17,
             "wide_rounds": -1}
    path.write_text(json.dumps({key: entry, "other@x": entry}))
    sc = fpt.Scene(scene)
    got = autotune.autotune("probe", scene=sc, run=run, cache_path=str(path), measure=False)
    assert got == entry
    assert autotune.autotune("absent", scene=sc, run=run, cache_path=str(path),
                             measure=False) is None
    best = autotune.autotune("measured", scene=sc, run=run, cache_path=str(path))
    assert best["ms"] > 0 and best["block_threads"] in (128, 256)
    cache = json.loads(path.read_text())
    assert set(cache) == {key, "other@x", "measured@" + autotune.device_tag()}
    assert cache[key] == entry
    path.write_text("{ not json")
    with pytest.raises(fpt.FptError):
        autotune.autotune("probe", scene=sc, run=run, cache_path=str(path), measure=False)
    sc.close()
