"""Refractive body boundaries on the oracle: a body medium of index n != 1
(the paper's glass beads and vials hold refractive media) has a smooth
dielectric boundary with vacuum.  A beam entering it and every path reaching
it from inside are reflected specularly with the unpolarised Fresnel
reflectance (1 beyond the critical angle), else cross it (Snell's law on
entry).  Pinned against closed forms of non-scattering absorbing slabs and
spheres, whose reflectance sequences can be summed exactly, and against the
index-matched walk at n = 1."""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from stats import binom_z, check_z, multinomial_z


def escape_fractions(scene, n_paths, seed=1):
    out = oracle.render(scene, workloads.make_run(n_paths, seed=seed))
    f = out["film"][0].sum(axis=(0, 2))       # [side] summed over components and bins
    return f[0], f[1], oracle.tallies_dict(out["tallies"])


def test_fresnel_reference_values():
    """The closed forms' Fresnel function against textbook values: normal
    incidence ((n-1)/(n+1))^2, Brewster's angle (R_p = 0, so R = R_s/2 =
    ((n^2-1)/(n^2+1))^2 / 2), total reflection from the critical angle on,
    grazing incidence 1, reciprocity R(ti, n1->n2) = R(tt, n2->n1), and no
    interface at all for n1 = n2."""
    for n in (1.33, 1.5, 2.4):
        assert cf.fresnel_unpolarised(1.0, 1.0, n) == pytest.approx(((n - 1) / (n + 1)) ** 2, rel=1e-12)
        cb = math.cos(math.atan(n))
        assert cf.fresnel_unpolarised(cb, 1.0, n) == pytest.approx(((n * n - 1) / (n * n + 1)) ** 2 / 2,
                                                                   rel=1e-9)
        tc = math.asin(1.0 / n)
        assert cf.fresnel_unpolarised(math.cos(tc) - 1e-9, n, 1.0) == 1.0
        assert cf.fresnel_unpolarised(math.cos(tc) + 1e-6, n, 1.0) > 0.98
        assert cf.fresnel_unpolarised(1e-7, 1.0, n) > 0.9999
        for ti in np.linspace(0.05, 1.5, 12):
            tt = math.asin(math.sin(ti) / n)
            assert cf.fresnel_unpolarised(math.cos(ti), 1.0, n) == pytest.approx(
                cf.fresnel_unpolarised(math.cos(tt), n, 1.0), rel=1e-10)
        assert cf.fresnel_unpolarised(0.3, n, n) == 0.0


@pytest.mark.parametrize("ior,theta", [(1.5, 0.0), (1.5, 30.0), (1.33, 60.0), (1.5, 80.0),
                                       (2.4, 45.0)])
def test_dielectric_slab_beam(ior, theta):
    """Beam into a non-scattering absorbing slab (sigma_a 0.5/mm, 1 mm) at
    oblique incidence: reflected and transmitted fractions, and the number of
    Fresnel reflections per path, r + (1-r) r q / (1 - r q), against the
    multiple-reflection sums."""
    n = 1 << 17
    R, T, t = escape_fractions(workloads.t9_dielectric_slab_beam(ior, theta), n)
    ci = math.cos(math.radians(theta))
    Rc, Tc = cf.dielectric_slab_beam(ior, ci, 0.5, 1.0)
    z = multinomial_z([R, T, 1 - R - T], n, [Rc, Tc, 1 - Rc - Tc])
    assert np.all(np.abs(z) < 4.5), (R, Rc, T, Tc, z)
    r = cf.fresnel_unpolarised(ci, 1.0, ior)
    q = math.exp(-0.5 / math.sqrt(1 - (1 - ci * ci) / ior ** 2))
    expect = r + (1 - r) * r * q / (1 - r * q)
    # per-path reflection counts are 0, 1, 2, ...: their variance is below the mean times 3
    assert abs(t["wall_reflect"] / n - expect) < 5 * math.sqrt(3 * expect / n) + 1e-9
    assert t["exit_excscat"] == 0 and t["scatters"] == 0


def test_dielectric_slab_point_source_with_total_reflection():
    """Isotropic source at 0.3 mm in a 1 mm slab of index 1.4 (critical angle
    45.6 degrees: 70 % of the directions are trapped until absorbed): bottom and
    top escape fractions against the quadrature over direction cosines."""
    n = 1 << 17
    bot, top, _ = escape_fractions(workloads.t10_dielectric_slab_point(1.4), n, seed=2)
    b, t = cf.dielectric_slab_point(1.4, 0.3, 1.0, 0.3)
    z = multinomial_z([bot, top, 1 - bot - top], n, [b, t, 1 - b - t])
    assert np.all(np.abs(z) < 4.5), (bot, b, top, t)


def test_dielectric_sphere_point_source():
    """Isotropic source at 0.8 of the radius from the centre of a sphere of
    index 1.5 (sigma_a 0.5/mm, radius 1 mm): chords with impact parameter above
    r/1.5 are trapped; the escape fraction against the quadrature over the
    emission angle."""
    n = 1 << 17
    bot, top, t = escape_fractions(workloads.t11_dielectric_sphere_point(1.5), n, seed=3)
    p = cf.dielectric_sphere_point(1.5, 0.5, 1.0, 0.8)
    assert abs(binom_z(round((bot + top) * n), n, p)) < 4.5, (bot + top, p)
    assert t["wall_reflect"] > 0


def test_index_matched_is_the_plain_walk():
    """n = 1 is no interface: every path of a scattering dye slab and a sphere
    body is the index-matched walk, record for record."""
    for scene in (workloads.slab_scene(), workloads.sphere_scene()):
        run = workloads.make_run(1 << 12, seed=4)
        a = oracle.render(scene, run, records=True)
        s1 = workloads.deepcopy(scene)
        s1["media"][0]["ior"] = 1.0
        b = oracle.render(s1, run, records=True)
        assert np.array_equal(a["records"].view(np.uint8), b["records"].view(np.uint8))
        assert np.array_equal(a["film"], b["film"])


def test_scattering_dielectric_slab_loses_no_path():
    """A conservative scattering slab (sigma_s 5/mm, n 1.5): every path leaves
    through one face or the scatter cap; internal reflections occur, and
    trapped directions are freed by the next scatter."""
    scene = workloads.t9_dielectric_slab_beam(1.5, 20.0, sigma_a=0.0, sigma_s=5.0)
    n = 1 << 14
    out = oracle.render(scene, workloads.make_run(n, seed=5))
    t = oracle.tallies_dict(out["tallies"])
    assert t["exit_esc_r"] + t["exit_esc_t"] + t["exit_scap"] == n
    assert t["exit_scap"] == 0
    assert t["wall_reflect"] > n
    R = out["film"][0, 0, 0].sum()
    # a mismatched boundary keeps light in longer but cannot create or destroy it
    assert abs(R + out["film"][0, 0, 1].sum() - 1.0) < 1e-12


def test_refractive_slab_gradients_match_finite_differences():
    """The path-replay gradient needs nothing new at a refracting boundary
    (the Fresnel decisions do not depend on concentration, QY or sigma_s): on
    a scattering dye slab behind water (n 1.33) the estimator of d<g, film>
    agrees with central differences of the walk under common random numbers."""
    B = 32
    n = 1 << 17
    rng = np.random.default_rng(9)

    def scene_fn(theta):
        s = workloads.slab_scene(sigma_s=theta[2], conc_uM=theta[0], qy=theta[1])
        s["media"][0]["ior"] = 1.33
        return s

    theta = [30.0, 0.7, 5.0]
    s = scene_fn(theta)
    run = workloads.make_run(n, seed=10, parity_batches=B)
    # transmission weighted over reflection: scattering moves light between the
    # faces, so sigma_s moves this functional (a uniform weight barely sees it)
    g = rng.random(oracle.film_shape(s, B)[1:])
    g[:, 1, :] += 2.0
    g = np.broadcast_to(g, oracle.film_shape(s, B)).copy()
    o = oracle.render(s, run, grad_film=g / B, record_grad=True)
    assert oracle.tallies_dict(o["tallies"])["wall_reflect"] > 0
    pg = o["record_grad"]
    per_batch = np.stack([pg[b::B].sum(0) for b in range(B)])
    z = []
    for i in range(3):
        h = 0.02
        tp, tm = list(theta), list(theta)
        tp[i] *= 1 + h
        tm[i] *= 1 - h
        fp = oracle.render(scene_fn(tp), run)["film"]
        fm = oracle.render(scene_fn(tm), run)["film"]
        fd = ((fp - fm) * g).reshape(B, -1).sum(1) / (2 * h * theta[i])
        est = per_batch[:, i] * B
        se_est = math.sqrt(est.var(ddof=1) / B)
        assert abs(est.mean()) > 3 * se_est, ("gradient not resolved", i)
        z.append((est.mean() - fd.mean()) / math.sqrt(est.var(ddof=1) / B + fd.var(ddof=1) / B))
    check_z(z, "refractive slab gradient vs central differences", dof=B - 1)
