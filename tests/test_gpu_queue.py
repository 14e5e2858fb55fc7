"""The path queue, camera connections and launch timing on the GPU: small and
ragged path counts (empty queue shards), a box scene with an escape sensor
(no camera work at all), and the library's launch timing."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from replay import compare_records
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
    o = oracle.render(scene, run, records=True)["records"]
    compare_records(rec, o, scale=1.0, sigma_t_max=200.0)


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
