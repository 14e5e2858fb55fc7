"""The descriptor maxima on the GPU (needs an MI355X).

A box at every maximum the ABI allows (8 spheres and media, 8 dyes with 4 in
every medium, 8 light lines, a 16-term spectrum) replays against the oracle
in both estimators; 1024 bins (the largest grid) replay on a slab and a box
and run batched, where the library fits the launch to the 160 KiB of LDS a
workgroup may hold; a scene whose tables cannot fit is refused before any
launch."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from replay import compare_records, oracle_replay

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _fpt():
    import paper_1706_03024_amd as fpt
    return fpt


def _tables_match(sc, scene):
    g = sc.tables()
    o = oracle.tables(scene)
    np.testing.assert_allclose(g["sigma_t"], o["sigma_t"].astype(np.float32), rtol=2.4e-7)
    np.testing.assert_allclose(g["emis_cdf"], o["emis_cdf"].astype(np.float32), rtol=2.4e-7,
                               atol=1e-30)
    if scene["geometry"]["kind"] == "box":
        np.testing.assert_allclose(g["rho"], o["rho"].astype(np.float32), rtol=2.4e-7)
    np.testing.assert_array_equal(g["line_bin"], o["line_bin"])


def test_maximal_box_scene():
    """Every maximum at once: tables, 2^14 forward paths and a full 1-sample
    camera-side render (16x16 pixels x 101 bins) replay against the oracle;
    the forward film equals the sum of the paths' deposits; the adjoint is
    refused (48 parameters over the 16 it carries)."""
    import torch
    fpt = _fpt()
    scene = workloads.maximal_scene()
    sc = fpt.Scene(scene)
    _tables_match(sc, scene)
    run = workloads.make_run(1 << 14, seed=91)
    t = fpt.new_tallies()
    film = sc.render(run, tallies=t)
    rec, _ = sc.records(run)
    torch.cuda.synchronize()
    print(compare_records(rec, oracle_replay(scene, run)))
    total = float(film.double().sum())
    assert total > 0.0
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    tal = fpt.tallies_dict(t)
    assert tal["emissions"] > 0 and tal["crossings"] > 0 and tal["exit_light"] > 0
    crun = workloads.make_run(oracle.camera_paths(scene, 1), seed=92)
    crec = sc.camera_records(crun)
    print(compare_records(crec, oracle_replay(scene, crun, camera=True)))
    assert np.sum(crec["splat_sum"] > 0) > 100
    assert sc.n_params == 48
    with pytest.raises(fpt.FptError) as e:
        sc.render_adjoint(run, torch.zeros_like(film))
    assert e.value.status == fpt._abi.E_UNSUPPORTED
    sc.close()


def test_oversized_tables_refused_before_launch():
    """At 1024 bins the maximal box's table image (8 media x 4 dye thresholds
    per bin) needs ~220 KB of LDS: forward, records and camera-side calls
    return FPT_E_UNSUPPORTED and leave the film untouched."""
    import torch
    fpt = _fpt()
    sc = fpt.Scene(workloads.maximal_scene(n_bins=1024, width=8))
    run = workloads.make_run(4096, seed=1)
    film = sc.new_film()
    for call in (lambda: sc.render(run, film=film), lambda: sc.records(run),
                 lambda: sc.render_camera(workloads.make_run(8 * 8 * 1024, seed=2), film=film)):
        with pytest.raises(fpt.FptError) as e:
            call()
        assert e.value.status == fpt._abi.E_UNSUPPORTED
        assert "LDS" in str(e.value)
    torch.cuda.synchronize()
    assert float(film.abs().sum()) == 0.0
    sc.close()


def test_maximum_bins_slab_and_box():
    """1024 bins: a dye slab (2^14 paths) and the three-sphere box (2^13
    forward paths, 4096 camera-side paths) replay against the oracle."""
    fpt = _fpt()
    slab = workloads.slab_scene(n_bins=1024)
    sc = fpt.Scene(slab)
    _tables_match(sc, slab)
    run = workloads.make_run(1 << 14, seed=93)
    rec, _ = sc.records(run)
    sc.close()
    print(compare_records(rec, oracle_replay(slab, run)))
    assert np.sum(rec["n_emit"] > 0) > 0

    box = workloads.cornell_scene(16, 16, n_bins=1024)
    sc = fpt.Scene(box)
    _tables_match(sc, box)
    run = workloads.make_run(1 << 13, seed=94)
    rec, _ = sc.records(run, max_vertices=512)
    print(compare_records(rec, oracle_replay(box, run, max_vertices=512)))
    n = oracle.camera_paths(box, 1)
    sub = workloads.make_run(4096, seed=95, path_begin=n // 2, total_paths=n)
    crec = sc.camera_records(sub, max_vertices=512)
    print(compare_records(crec, oracle_replay(box, sub, max_vertices=512, camera=True)))
    sc.close()


def test_maximum_bins_batch_equals_standalone():
    """Batched slabs at 1024 bins: a wave's slot (tables and histogram, 53 KB)
    does not fit four times in a workgroup's LDS, so the launch takes fewer
    waves per block; every instance is still bit-identical to its standalone
    render."""
    import torch
    fpt = _fpt()
    scenes = [workloads.slab_scene(n_bins=1024, conc_uM=c, sigma_s=s)
              for c, s in ((5.0, 10.0), (20.0, 4.0), (2.0, 30.0))]
    runs = [workloads.make_run(1 << 14, seed=96 + i, instance=i) for i in range(len(scenes))]
    b = fpt.Batch(scenes, runs)
    films = b.new_films()
    tal = fpt.new_tallies(len(scenes))
    b.render(films, tal)
    torch.cuda.synchronize()
    for i, (s, r) in enumerate(zip(scenes, runs)):
        sc = fpt.Scene(s)
        t = fpt.new_tallies()
        f = sc.render(r, tallies=t)
        torch.cuda.synchronize()
        assert torch.equal(f[0], films[i]), f"instance {i}"
        assert torch.equal(t, tal[i]), f"instance {i} tallies"
        sc.close()
    b.close()
