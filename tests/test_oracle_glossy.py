"""Pins of the oracle's glossy walls (sec. 5, the glossy Cornell box): a
normalised modified-Phong lobe rho (n+2)/(2 pi) cos^n(alpha) about the mirror
direction, sampled about the mirror direction with a per-path throughput
weight.

* White furnace: at normal incidence the lobe's directional albedo over rho is
  exactly 1 (the (n+2)/(2 pi) normalisation), at oblique incidence the
  quadrature of the lobe clipped by the wall; the sampler's mean throughput
  factor equals it.
* Reciprocity: lobe(wi -> wo) = lobe(-wo -> -wi).
* The sampler's directions follow the lobe: weighted moments of the sampled
  directions equal the lobe's moments by quadrature.
* First-bounce radiance: a glossy back wall lit only by the quad light reads
  rho int lobe L cos cos / r^2 dA over the light, by quadrature, pixel by
  pixel (batch means).
* Planted mistakes in the test's own model (an unnormalised lobe, the lobe
  about the normal instead of the mirror direction) fail the radiance check.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from stats import check_z
from test_oracle_camera_pins import B, _batches, _camera, _classify

N_UP = np.array([0.0, 0.0, 1.0])


def _incoming(theta_deg, phi_deg=30.0):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return -np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


def _grid_samples(n, wi, k=256):
    u = (np.arange(k) + 0.5) / k
    wo, f = [], []
    for a in u:
        for b in u:
            w, x = oracle.phong_sample(n, wi, N_UP, a, b)
            wo.append(w)
            f.append(x)
    return np.array(wo), np.array(f)


@pytest.mark.parametrize("n", [1.0, 20.0, 200.0])
def test_white_furnace(n):
    normal_albedo = cf.hemisphere_integral(
        lambda w: np.array([[oracle.phong_eval(n, _incoming(0.0), x, N_UP) for x in row] for row in w]),
        N_UP, n_theta=128, n_phi=64)
    assert abs(normal_albedo - 1.0) < 2e-4
    for th in (0.0, 45.0, 75.0):
        wi = _incoming(th)
        albedo = cf.hemisphere_integral(lambda w: cf.phong_lobe(n, wi, w, N_UP), N_UP)
        wo, f = _grid_samples(n, wi, k=128)
        assert np.all(f >= 0.0) and np.all((f > 0) == (wo @ N_UP > 0))
        assert abs(f.mean() - albedo) < 3e-3 * albedo + 1e-4, (n, th, f.mean(), albedo)
        if th == 0.0:
            assert abs(albedo - 1.0) < 2e-3
        else:
            assert albedo < 1.0


def test_reciprocity():
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = rng.normal(size=3), rng.normal(size=3)
        wi = a / np.linalg.norm(a)
        wo = b / np.linalg.norm(b)
        if wi @ N_UP > 0:
            wi = -wi
        if wo @ N_UP < 0:
            wo = -wo
        n = rng.uniform(0.5, 100.0)
        f1 = oracle.phong_eval(n, wi, wo, N_UP)
        f2 = oracle.phong_eval(n, -wo, -wi, N_UP)
        assert abs(f1 - f2) <= 1e-12 * max(f1, 1e-300)
        assert abs(f1 - float(cf.phong_lobe(n, wi, wo, N_UP))) <= 1e-12 * max(f1, 1e-300)


@pytest.mark.parametrize("n,th", [(5.0, 30.0), (50.0, 60.0)])
def test_sampled_directions_follow_the_lobe(n, th):
    wi = _incoming(th)
    wo, f = _grid_samples(n, wi, k=192)
    for g in (lambda w: w[..., 0] ** 2, lambda w: w[..., 1] * w[..., 2] + 1.0, lambda w: w[..., 2] ** 3):
        est = float(np.mean(f * g(wo)))
        ref = cf.hemisphere_integral(lambda w: cf.phong_lobe(n, wi, w, N_UP) * g(w), N_UP)
        assert abs(est - ref) < 4e-3 * abs(ref) + 1e-4, (n, th, est, ref)


def _glossy_back_wall(n_exp, rho, W):
    s = workloads.dark_box_scene(width=W, height=W, lines=[(550, 1.0)])
    s["geometry"]["walls"][4] = workloads.pwl((300, rho), (800, rho))
    s["geometry"]["wall_gloss"] = [0.0, 0.0, 0.0, 0.0, n_exp, 0.0]
    return s


@pytest.mark.parametrize("n_exp", [4.0, 30.0])
def test_first_bounce_glossy_wall_radiance(n_exp):
    W, rho = 24, 0.6
    s = _glossy_back_wall(n_exp, rho, W)
    cam = _camera(s)
    film = _batches(s, 1 << 19, seed=7)
    li = s["light"]
    corner, u, v = (np.array(li[k], float) for k in ("corner", "u", "v"))
    Le = 1.0 / (math.pi * 0.25)
    rows = []
    for py in range(W):
        for px in range(W):
            if any(k != "wall4" for k, _, _ in _classify(s, cam, px, py, corners=True)):
                continue
            cls = _classify(s, cam, px, py, sub=3)
            g, wg = np.polynomial.legendre.leggauss(3)
            wts = np.outer(wg, wg).ravel() / 4.0
            Ls, Lw = [], []
            for _, q, d in cls:
                we = -np.asarray(d) / np.linalg.norm(d)
                Ls.append(cf.glossy_wall_radiance(q, N_UP, we, corner, u, v, Le, rho, n_exp))
                # planted mistakes: the lobe without its (n+2)/2 normalisation,
                # and the lobe about the normal instead of the mirror direction
                Lw.append((Ls[-1] * 2.0 / (n_exp + 2.0),
                           cf.glossy_wall_radiance(q, N_UP, we, corner, u, v, Le, rho, n_exp,
                                                   about_normal=True)))
            vals = film[:, 0, py, px, 50]
            rows.append((vals.mean(), vals.std(ddof=1) / math.sqrt(B), float(np.dot(wts, Ls)),
                         [float(np.dot(wts, [w[k] for w in Lw])) for k in range(2)]))
    # pixels far in the lobe's tail (expected radiance below 1e-4 of the
    # brightest: cos^n(alpha) of 1e-11 and less) get their value from rare
    # samples, whose batch means are too heavy-tailed for a z-test
    top = max(r[2] for r in rows)
    z = [(m - e) / se for m, se, e, _ in rows if e >= 1e-4 * top]
    assert len(z) >= 20
    check_z(z, f"first-bounce glossy wall radiance n={n_exp}", dof=B - 1)
    for k, name in enumerate(("unnormalised lobe", "lobe about the normal")):
        z_wrong = [(m - w[k]) / se for m, se, e, w in rows if e >= 1e-4 * top]
        with pytest.raises(AssertionError):
            check_z(z_wrong, "planted: " + name, dof=B - 1)


def test_glossy_walls_need_a_pinhole_and_the_forward_walk():
    s = workloads.slab_scene()
    box = workloads.cornell_scene(8, 8)
    box["sensor"] = {"kind": "escape"}
    box["geometry"]["wall_gloss"] = [0.0, 0.0, 10.0, 0.0, 0.0, 0.0]
    with pytest.raises(oracle.OracleError):
        oracle.render(box, workloads.make_run(16))
    cam = workloads.cornell_scene(8, 8)
    cam["geometry"]["wall_gloss"] = [0.0, 0.0, 10.0, 0.0, 0.0, 0.0]
    oracle.render(cam, workloads.make_run(16))
    with pytest.raises(oracle.OracleError):
        oracle.render_camera(cam, workloads.make_run(oracle.camera_paths(cam, 1)))
    del s
