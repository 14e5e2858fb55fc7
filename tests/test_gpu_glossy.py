"""Glossy walls on the GPU (the paper's glossy Cornell box, sec. 5) against the
oracle: per-path replay of the walk with its lobe-sampled directions and
weighted deposits, the film by batch means, the path-replay gradient, and the
forward instantiation's film against the replayed records on the same paths."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

import oracle
import workloads
from replay import check_grad_total, compare_records, oracle_replay
from stats import batch_z, check_z

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


@pytest.mark.parametrize("back,floor", [(30.0, 8.0), (200.0, 1.0)])
def test_glossy_replay(back, floor):
    """2^15 paths of a glossy Cornell box replay against the oracle: the same
    reflections, lobe directions, exits below the wall and weighted deposits."""
    scene = workloads.glossy_cornell_scene(32, 32, back=back, floor=floor)
    run = workloads.make_run(1 << 15, seed=71)
    sc = _fpt().Scene(scene)
    rec, _ = sc.records(run)
    sc.close()
    cond = oracle_replay(scene, run)
    print(compare_records(rec, cond))
    o = cond["records"]
    # paths whose lobe direction fell below a glossy wall end at it (exit WALL)
    assert np.sum(o["exit_code"] == 6) > 100


def test_glossy_film_and_identity():
    """The forward instantiation (weights in the deferred connection queue):
    the film in 32 parity slices agrees bin by bin with the oracle's film of
    independent paths, and on the same paths its total equals the sum of the
    replayed records' deposits; its tallies equal the oracle's up to marginal
    paths.  The allocation-free variant gives the same tallies."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd import _abi
    B = 32
    scene = workloads.glossy_cornell_scene(32, 32)
    sc = fpt.Scene(scene)
    g = sc.render(workloads.make_run(1 << 22, seed=72, parity_batches=B)).cpu().numpy().astype(np.float64)
    same = workloads.make_run(1 << 18, seed=73)
    t = fpt.new_tallies()
    film = sc.render(same, tallies=t)
    rec, _ = sc.records(same)
    t2 = fpt.new_tallies()
    film2 = sc.new_film()
    r = _abi.run_struct(same)
    _abi.check(_abi.lib().fpt_render_noalloc(sc.handle, C.byref(r), C.c_void_p(film2.data_ptr()),
                                             C.c_void_p(t2.data_ptr()),
                                             C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    total = float(film.double().sum())
    sc.close()
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    assert torch.equal(t, t2)
    np.testing.assert_allclose(film2.cpu().numpy(), film.cpu().numpy(), rtol=1e-5,
                               atol=1e-7 * float(film.max()))
    tg = fpt.tallies_dict(t)
    to = oracle.tallies_dict(oracle.render(scene, same)["tallies"])
    for k in ("vertices", "wall_reflect", "exit_wall", "splat_hit", "splat_miss"):
        assert abs(tg[k] - to[k]) <= max(8, 1e-4 * to[k]), (k, tg[k], to[k])
    # equal path counts on both sides: a glossy highlight's deposits are rare and
    # large (the lobe toward the eye reaches (n+2)/2), so a smaller oracle run
    # sees too few of them (measured: the oracle at 2^19 paths against itself at
    # 2^22 fails this test as the GPU does; at 2^22 both pass)
    o = oracle.render(scene, workloads.make_run(1 << 22, seed=74, parity_batches=B))["film"]
    z = batch_z(g, o)
    assert z.size > 500
    check_z(z, "glossy Cornell film: GPU vs oracle", dof=B - 1)


def test_glossy_adjoint_replay():
    """The path-replay gradient with weighted paths: per-path contributions and
    the reduced total against the oracle (the weights do not depend on the
    parameters, so the estimator is the plain walk's)."""
    import torch
    fpt = _fpt()
    scene = workloads.glossy_cornell_scene(16, 16)
    for m in range(3):
        scene["media"][m]["dyes"][0][1] *= 20
    run = workloads.make_run(1 << 14, seed=75)
    gfilm = 1.0 + np.random.default_rng(6).random(oracle.film_shape(scene))
    sc = fpt.Scene(scene)
    gt = torch.tensor(gfilm, dtype=torch.float32, device="cuda")
    rec, rg = sc.records(run, grad_film=gt)
    total = sc.render_adjoint(run, gt)
    torch.cuda.synchronize()
    sc.close()
    cond = oracle_replay(scene, run, grad_film=gfilm)
    print(compare_records(rec, cond, gpu_grad=rg))
    print("total deviations", check_grad_total(total.cpu().numpy(), rg, cond))


def test_camera_side_refuses_glossy_walls():
    import torch
    fpt = _fpt()
    scene = workloads.glossy_cornell_scene(8, 8)
    sc = fpt.Scene(scene)
    with pytest.raises(fpt.FptError) as e:
        sc.render_camera(workloads.make_run(oracle.camera_paths(scene, 1)))
    assert e.value.status == fpt._abi.E_UNSUPPORTED
    torch.cuda.synchronize()
    sc.close()
