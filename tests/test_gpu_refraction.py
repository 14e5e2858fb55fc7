"""GPU refractive body boundaries vs the oracle and the closed forms (needs an
MI355X): a body medium of index n != 1 reflects an entering beam and paths
reaching its boundary from inside with the unpolarised Fresnel reflectance
(total internal reflection beyond the critical angle), else lets them cross
(Snell's law on entry).  Replay on identical streams, escape fractions
against the multiple-reflection closed forms at 2^22 paths, and the batched
kernel against standalone renders."""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from replay import check_grad_total, compare_records, oracle_replay
from stats import binom_z, multinomial_z

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


def refractive_dye_slab(ior=1.33):
    s = workloads.slab_scene()
    s["media"][0]["ior"] = ior
    return s


def refractive_dye_sphere(ior=1.5):
    s = workloads.sphere_scene()
    s["media"][0]["ior"] = ior
    return s


SCENES = {
    "slab_beam_60deg": lambda: workloads.t9_dielectric_slab_beam(1.33, 60.0),
    "slab_point_tir": lambda: workloads.t10_dielectric_slab_point(1.4),
    "sphere_point_tir": lambda: workloads.t11_dielectric_sphere_point(1.5),
    "dye_slab_water": refractive_dye_slab,
    "dye_sphere_glass": refractive_dye_sphere,
}


@pytest.mark.parametrize("name", sorted(SCENES))
def test_refractive_replay(name):
    """2^14 paths per scene replay against the oracle: Fresnel decisions,
    total internal reflections and refracted entries land on the same
    vertices, exits and states."""
    scene = SCENES[name]()
    run = workloads.make_run(1 << 14, seed=61)
    fpt = _fpt()
    sc = fpt.Scene(scene)
    rec, _ = sc.records(run)
    sc.close()
    rep = compare_records(rec, oracle_replay(scene, run))
    print(name, rep)


def _escape(scene, n, seed):
    import torch
    fpt = _fpt()
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    film = sc.render(workloads.make_run(n, seed=seed), tallies=t)
    torch.cuda.synchronize()
    f = film.cpu().numpy().astype(np.float64)[0].sum(axis=(0, 2))
    sc.close()
    return f[0], f[1], fpt.tallies_dict(t)


@pytest.mark.parametrize("ior,theta", [(1.5, 0.0), (1.33, 60.0), (1.5, 80.0), (2.4, 45.0)])
def test_gpu_dielectric_slab_beam(ior, theta):
    n = 1 << 22
    R, T, t = _escape(workloads.t9_dielectric_slab_beam(ior, theta), n, 62)
    Rc, Tc = cf.dielectric_slab_beam(ior, math.cos(math.radians(theta)), 0.5, 1.0)
    z = multinomial_z([R, T, 1 - R - T], n, [Rc, Tc, 1 - Rc - Tc])
    assert np.all(np.abs(z) < 4.5), (R, Rc, T, Tc)
    assert t["paths"] == n


def test_gpu_dielectric_point_sources():
    n = 1 << 22
    bot, top, _ = _escape(workloads.t10_dielectric_slab_point(1.4), n, 63)
    b, t = cf.dielectric_slab_point(1.4, 0.3, 1.0, 0.3)
    z = multinomial_z([bot, top, 1 - bot - top], n, [b, t, 1 - b - t])
    assert np.all(np.abs(z) < 4.5), (bot, b, top, t)
    bot, top, _ = _escape(workloads.t11_dielectric_sphere_point(1.5), n, 64)
    p = cf.dielectric_sphere_point(1.5, 0.5, 1.0, 0.8)
    assert abs(binom_z(round((bot + top) * n), n, p)) < 4.5, (bot + top, p)


def test_refractive_batch_equals_standalone():
    """Refractive instances in the batched kernel are bit-identical to their
    standalone renders (integer escape tallies, same keys)."""
    import torch
    fpt = _fpt()
    scenes = [refractive_dye_slab(1.33), refractive_dye_sphere(1.5),
              workloads.t9_dielectric_slab_beam(1.5, 30.0, sigma_s=2.0),
              workloads.t10_dielectric_slab_point(2.0, sigma_s=1.0)]
    runs = [workloads.make_run(1 << 14, seed=70 + i, instance=i) for i in range(len(scenes))]
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
        assert fpt.tallies_dict(t)["wall_reflect"] > 0
        sc.close()
    b.close()


@pytest.mark.parametrize("make", [refractive_dye_slab, refractive_dye_sphere])
def test_refractive_adjoint_replay(make):
    """The adjoint's refracting instantiation: each path's gradient
    contribution matches the oracle's (same streams), and the reduced
    gradient equals the sum of the contributions and the oracle's total."""
    import torch
    fpt = _fpt()
    scene = make()
    run = workloads.make_run(1 << 14, seed=81)
    rng = np.random.default_rng(4)
    g = rng.random(oracle.film_shape(scene))
    g[:, :, 1, :] += 2.0
    sc = fpt.Scene(scene)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    rec, rg = sc.records(run, grad_film=gt)
    total = sc.render_adjoint(run, gt)
    torch.cuda.synchronize()
    total = total.cpu().numpy().astype(np.float64)
    sc.close()
    cond = oracle_replay(scene, run, grad_film=g)
    assert np.sum(rec["exit_code"] <= 1) > 0
    print(compare_records(rec, cond, gpu_grad=rg))
    print("total deviations", check_grad_total(total, rg, cond))
