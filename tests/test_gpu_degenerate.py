"""Degenerate parameter values on the GPU vs the oracle (needs an MI355X):
quantum yields 0 and 1, a dye at zero concentration, scatter caps of 0 and 1,
unlimited emissions, and a batch with an instance that has no paths.  Each
case replays per path against the oracle, gradient contributions included
(the score terms 1/QY, 1/(1-QY) and 1/c are stored as 0 where their event
cannot happen)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from replay import compare_records, oracle_replay

pytestmark = pytest.mark.gpu

SCAP = 5   # exit code of the scatter cap


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


def _zero_conc_slab():
    s = workloads.slab_scene()
    s["media"][0]["dyes"] = [[0, 0.0]]
    return s


CASES = {
    "qy_0": (lambda: workloads.slab_scene(qy=0.0), {}),
    "qy_1": (lambda: workloads.slab_scene(qy=1.0), {}),
    "conc_0": (_zero_conc_slab, {}),
    "scatter_cap_0": (lambda: workloads.slab_scene(), {"max_scatter": 0}),
    "scatter_cap_1": (lambda: workloads.slab_scene(), {"max_scatter": 1}),
    "emissions_unlimited": (lambda: workloads.slab_scene(conc_uM=200.0, qy=0.95),
                            {"max_emissions": workloads.UNLIMITED_EMISSIONS}),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_degenerate_replay(case):
    import torch
    fpt = _fpt()
    make, kw = CASES[case]
    scene = make()
    run = workloads.make_run(1 << 14, seed=97, **kw)
    g = np.random.default_rng(5).random(oracle.film_shape(scene))
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    film = sc.render(run, tallies=t)
    rec, rg = sc.records(run, grad_film=torch.tensor(g, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    tal = fpt.tallies_dict(t)
    f = film.cpu().numpy()
    sc.close()
    o = oracle.render(scene, run, film=False)
    assert np.all(np.isfinite(rg))
    print(case, compare_records(rec, oracle_replay(scene, run, grad_film=g), gpu_grad=rg))
    to = oracle.tallies_dict(o["tallies"])
    n = run["path_count"]
    assert tal["paths"] == n
    # the case's defining outcome, on both sides
    if case == "qy_0":
        assert tal["emissions"] == to["emissions"] == 0 and tal["dye_abs"] > 0
        assert np.all(f[:, 1] == 0.0)
    elif case == "qy_1":
        assert tal["exit_nonrad"] == to["exit_nonrad"] == 0 and tal["emissions"] > 0
    elif case == "conc_0":
        assert tal["dye_abs"] == to["dye_abs"] == 0
    elif case.startswith("scatter_cap"):
        # the scatter that goes over the cap is counted and ends the path
        cap = kw["max_scatter"]
        assert rec["n_scatter"].max() == cap + 1 and tal["exit_scap"] > 0
        assert np.array_equal(rec["n_scatter"] == cap + 1, rec["exit_code"] == SCAP)
    else:
        assert rec["n_emit"].max() >= 10 and tal["exit_kcap"] == 0
    for k in ("exit_scap", "exit_nonrad", "exit_kcap", "emissions"):
        assert abs(tal[k] - to[k]) <= max(4, 1e-3 * to[k]), (k, tal[k], to[k])


def test_batch_with_an_instance_without_paths():
    """An instance whose run has no paths contributes nothing and disturbs no
    other instance (each bit-identical to its standalone render)."""
    import torch
    fpt = _fpt()
    scenes = [workloads.slab_scene(conc_uM=c) for c in (5.0, 10.0, 20.0)]
    runs = [workloads.make_run(1 << 14, seed=98, instance=0),
            dict(workloads.make_run(1 << 14, seed=98, instance=1), path_count=0),
            workloads.make_run(1 << 14, seed=98, instance=2)]
    b = fpt.Batch(scenes, runs)
    films = b.new_films()
    tal = fpt.new_tallies(3)
    b.render(films, tal)
    torch.cuda.synchronize()
    assert float(films[1].abs().sum()) == 0.0 and int(tal[1].abs().sum()) == 0
    for i in (0, 2):
        sc = fpt.Scene(scenes[i])
        t = fpt.new_tallies()
        f = sc.render(runs[i], tallies=t)
        torch.cuda.synchronize()
        assert torch.equal(f[0], films[i]) and torch.equal(t, tal[i]), i
        sc.close()
    b.close()
