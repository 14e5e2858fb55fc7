"""Batched form: one persistent launch over many instances, replayed from a
hipGraph, against standalone renders of the same instances and the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from stats import check_z, escape_z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _subset(n=48, max_paths=1 << 14):
    inst = workloads.load_batch_instances()[:n]
    for i in inst:
        i["paths"] = min(i["paths"], max_paths)
    return workloads.batch_config(inst)


def test_batched_instances_equal_standalone_renders():
    """Integer escape tallies make every instance of the batched launch
    bit-identical to the same instance rendered alone with the same key."""
    import torch
    import paper_1706_03024_amd as fpt
    scenes, runs = _subset()
    b = fpt.Batch(scenes, runs, tune={"chunk_paths": 1024})
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


def test_batched_graph_replays():
    """Replays of the captured graph, with eager work and synchronisation in
    between, give the same films as the first replay; a new film buffer is
    captured afresh."""
    import torch
    import paper_1706_03024_amd as fpt
    scenes, runs = _subset(32)
    b = fpt.Batch(scenes, runs)
    films = b.new_films()
    b.render(films)
    torch.cuda.synchronize()
    ref = films.clone()
    for _ in range(3):
        films.zero_()
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        b.render(films)
        torch.cuda.synchronize()
        assert torch.equal(films, ref)
    other = b.new_films()
    b.render(other)
    torch.cuda.synchronize()
    assert torch.equal(other, ref)
    b.render(other)  # accumulates
    torch.cuda.synchronize()
    assert torch.equal(other, 2 * ref)
    b.close()


def test_batched_vs_oracle_sampled():
    """A sample of instances at full path counts against the oracle with
    independent seeds (multinomial z-scores per bin)."""
    import torch
    import paper_1706_03024_amd as fpt
    inst = workloads.load_batch_instances()
    pick = [0, 5, 17, 100, 511, 1023]
    sub = [inst[i] for i in pick]
    scenes, runs = workloads.batch_config(sub)
    b = fpt.Batch(scenes, runs)
    films = b.new_films()
    b.render(films)
    torch.cuda.synchronize()
    g = films.cpu().numpy().astype(np.float64)
    b.close()
    z = []
    for k, (s, r) in enumerate(zip(scenes, runs)):
        n_o = min(r["path_count"], 1 << 13)
        o = oracle.render(s, dict(r, seed=77, path_count=n_o, total_paths=n_o))
        z.append(escape_z(g[k], r["path_count"], o["film"][0], n_o))
    check_z(np.concatenate(z), "batched instances vs oracle")


def _bench_shape(scenes, runs):
    """The batch in the launch shape the benchmark times (the cached tune)."""
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import autotune
    b = fpt.Batch(scenes, runs)
    tune = autotune.autotune("batched-1024", batch=b, measure=False)
    if tune is None:
        return b
    b.close()
    return fpt.Batch(scenes, runs, tune={k: v for k, v in tune.items() if k != "ms"})


def test_full_batch_runs_and_conserves():
    """The full 1024-instance workload in one graph launch, in the benchmark's
    launch shape: every instance's exits add up to its path count, and three
    instances are bit-identical to their standalone renders."""
    import torch
    import paper_1706_03024_amd as fpt
    scenes, runs = workloads.batch_config()
    b = _bench_shape(scenes, runs)
    films = b.new_films()
    tal = fpt.new_tallies(len(scenes))
    b.render(films, tal)
    torch.cuda.synchronize()
    t = tal.cpu().numpy()
    paths = np.array([r["path_count"] for r in runs])
    np.testing.assert_array_equal(t[:, 0], paths)
    np.testing.assert_array_equal(t[:, 10:20].sum(1), paths)
    f = films.cpu().numpy().astype(np.float64)
    esc = (t[:, 10] + t[:, 11]) / paths
    np.testing.assert_allclose(f.sum((1, 2, 3)), esc, rtol=1e-5, atol=1e-6)
    b.close()
    for i in (0, 511, 1023):
        sc = fpt.Scene(scenes[i])
        ti = fpt.new_tallies()
        fi = sc.render(runs[i], tallies=ti)
        torch.cuda.synchronize()
        assert torch.equal(fi[0], films[i]) and torch.equal(ti, tal[i]), i
        sc.close()


def test_autotune_returns_a_valid_shape():
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import autotune
    scene, run = workloads.slab_config()
    sc = fpt.Scene(scene)
    best = autotune.autotune("test-slab", scene=sc, run=run, cache_path="/tmp/fpt_tune_test.json",
                             force=True)
    assert best["block_threads"] in (128, 256) and best["ms"] > 0
    sc.close()
