"""The oracle's camera-side estimator (sec. 4.1: paths start at the camera at
the emission wavelength and sample the light only where an emission is
realised; sec. 4.3, eq. 12), pinned against the forward light walk.

With excitation scattering switched off (a path that has not emitted ends at
its first scatter or wall reflection) and K = 1, the forward walk's emitted
component estimates exactly what the camera-side estimator estimates: direct
excitation from the light, one re-emission, full transport at the emission
wavelength.  The two share the scene tables and nothing of the walk, so a
dropped factor on either side (1/4pi, the emitter cosine, a line weight, the
transmittance at the excitation wavelength, the pinhole importance) shows up
as a bias between them."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from stats import check_z


def direct_scene(width=8, n_bins=26):
    """The three-sphere Cornell box with lighter scattering and denser dye, so
    that direct excitation is common enough for the forward walk."""
    s = workloads.cornell_scene(width=width, height=width, n_bins=n_bins,
                                conc_scale=(4.0, 4.0, 40.0))
    for m, ss in zip(s["media"], (2.0, 4.0, 8.0)):
        m["sigma_s"] = ss
    return s


def shadow_scene(width=8, n_bins=26):
    """Off-axis geometry: a dye sphere high on the right, seen from the
    ceiling light at about 55 degrees, partly shadowed by a small absorbing
    sphere on the way; a second dye sphere low on the left."""
    s = direct_scene(width, n_bins)
    s["media"] = [
        {"sigma_s": 3.0, "sigma_a_bg": 0.01, "dyes": [[0, 200.0]]},
        {"sigma_s": 5.0, "sigma_a_bg": 0.01, "dyes": [[1, 40.0]]},
        {"sigma_s": 0.0, "sigma_a_bg": 30.0, "dyes": []},
    ]
    s["geometry"]["spheres"] = [
        {"center": [0.6, 0.45, 0.0], "radius": 0.3, "medium": 0},
        {"center": [-0.5, -0.6, 0.2], "radius": 0.3, "medium": 1},
        {"center": [0.28, 0.78, 0.0], "radius": 0.12, "medium": 2},
    ]
    return s


def slice_z(a, b):
    """z of the difference of two per-slice estimates (axis 0 = slice)."""
    B = a.shape[0]
    ma, mb = a.mean(0), b.mean(0)
    va, vb = a.var(0, ddof=1) / B, b.var(0, ddof=1) / B
    return (ma - mb) / np.sqrt(va + vb), ma, mb


def camera_run(scene, spp, seed, B=1, **kw):
    n = oracle.camera_paths(scene, spp)
    return workloads.make_run(n, seed=seed, parity_batches=B, **kw)


@pytest.mark.parametrize("make_scene", [direct_scene, shadow_scene])
def test_camera_side_matches_forward_direct_excitation(make_scene):
    sc = make_scene()
    B = 16
    fwd = oracle.render(sc, workloads.make_run(1 << 23, seed=11, excitation_scatter=False,
                                                max_emissions=1, parity_batches=B))
    cam = oracle.render_camera(sc, camera_run(sc, 256, seed=12, B=B))
    ff, fc = fwd["film"][:, 1], cam["film"][:, 1]   # [B][H][W][N]
    assert np.all(cam["film"][:, 0] == 0.0)
    z, ma, mb = slice_z(ff.sum(axis=(1, 2, 3)), fc.sum(axis=(1, 2, 3)))
    assert abs(z) < 4.0, (ma, mb, z)
    assert mb > 0.0
    z, ma, mb = slice_z(ff.sum(axis=(1, 2)), fc.sum(axis=(1, 2)))
    keep = mb > 1e-2 * mb.max()   # bins the forward walk samples at all
    assert keep.sum() >= 10
    check_z(z[keep], "spectrum", dof=B - 1)
    z, ma, mb = slice_z(ff.sum(axis=3), fc.sum(axis=3))
    keep = mb > 1e-2 * mb.max()
    check_z(z[keep], "image", dof=B - 1)


def test_camera_side_is_linear_in_quantum_yield():
    """QY enters only the source term, never a decision of the walk: halving
    it halves every deposit and leaves the walk unchanged."""
    sc = direct_scene(width=6, n_bins=11)
    run = camera_run(sc, 4, seed=3)
    a = oracle.render_camera(sc, run, records=True)
    half = workloads.deepcopy(sc)
    for d in half["dyes"]:
        d["qy"] *= 0.5
    b = oracle.render_camera(half, run, records=True)
    assert a["film"].sum() > 0.0
    np.testing.assert_allclose(b["film"], 0.5 * a["film"], rtol=1e-12, atol=0.0)
    assert np.array_equal(a["tallies"], b["tallies"])
    assert np.array_equal(a["records"]["exit_code"], b["records"]["exit_code"])


def test_camera_side_slices_average_to_the_whole():
    """Path p goes to slice s % B with weight B/spp: the slices' mean is the
    unsliced film, path by path."""
    sc = direct_scene(width=4, n_bins=11)
    one = oracle.render_camera(sc, camera_run(sc, 8, seed=5))
    four = oracle.render_camera(sc, camera_run(sc, 8, seed=5, B=4))
    np.testing.assert_allclose(four["film"].mean(axis=0), one["film"][0], rtol=1e-12,
                               atol=1e-300)
    assert np.array_equal(one["tallies"], four["tallies"])


def test_camera_side_path_layout():
    """p = ((s*H + py)*W + px)*N + k: a range of N paths covers one pixel at
    every bin, and deposits land in that pixel only."""
    sc = direct_scene(width=8, n_bins=11)
    W, N = 8, 11
    px, py = 3, 5                       # a pixel that sees the middle sphere
    run = camera_run(sc, 64, seed=9)
    total = run["total_paths"]
    film = np.zeros(oracle.film_shape(sc))
    recs = []
    for s in range(64):
        r = dict(run, path_begin=((s * W + py) * W + px) * N, path_count=N,
                 total_paths=total)
        out = oracle.render_camera(sc, r, records=True)
        film += out["film"]
        recs.append(out["records"])
    rec = np.concatenate(recs)
    assert np.array_equal(rec["lambda"], np.tile(np.arange(N), 64))
    assert np.all(rec["comp"] == 1) and np.all(rec["n_emit"] == 0)
    mask = np.zeros(film.shape, bool)
    mask[0, 1, py, px, :] = True
    assert np.all(film[~mask] == 0.0)
    assert film[mask].sum() > 0.0
    np.testing.assert_allclose(film[mask].sum(), rec["splat_sum"].sum(), rtol=1e-12)


def test_camera_side_without_dye_or_light_faces_is_dark():
    """A scattering sphere without dye has no source: nothing is deposited and
    no light connection is made; the walk itself still runs."""
    medium = {"sigma_s": 5.0, "sigma_a_bg": 0.1, "dyes": []}
    sc = workloads.dark_box_scene(sphere_medium=medium, width=8, height=8, n_bins=11,
                                  wall_rho=0.5)
    out = oracle.render_camera(sc, camera_run(sc, 2, seed=1))
    t = oracle.tallies_dict(out["tallies"])
    assert np.all(out["film"] == 0.0)
    assert t["splat_hit"] == 0 and t["splat_miss"] == 0
    assert t["scatters"] > 0 and t["wall_reflect"] > 0
    assert t["paths"] == oracle.camera_paths(sc, 2)
    exits = sum(v for k, v in t.items() if k.startswith("exit_"))
    assert exits == t["paths"]
    assert t["exit_nonrad"] == 0 and t["exit_excscat"] == 0


def test_camera_side_eye_rays_enter_through_the_open_face():
    """The pinhole sits 3.4 in front of the open z = +1 face with a 40 degree
    field: the ray through pixel centre (px, py) misses the box exactly when
    its crossing of z = 1 lies outside [-1, 1]^2 (checked on pixels whose
    crossing is far from an edge)."""
    sc = workloads.dark_box_scene(width=16, height=16, n_bins=3)
    W = H = 16
    run = camera_run(sc, 1, seed=2)
    out = oracle.render_camera(sc, run, records=True, max_vertices=1)
    rec = out["records"]
    t = np.tan(np.radians(20.0))
    for p in range(run["total_paths"]):
        pix = p // 3
        px, py = pix % W, pix // W
        xi = 2.0 * (px + 0.5) / W - 1.0
        yi = 1.0 - 2.0 * (py + 0.5) / H
        # crossing of z = 1 from the eye at z = 3.4 looking along -z
        qx, qy = 2.4 * xi * t, 2.4 * yi * t
        slack = 2.4 * t * 2.0 / W       # a pixel's width at that depth
        inside = max(abs(qx), abs(qy)) < 1.0 - slack
        outside = max(abs(qx), abs(qy)) > 1.0 + slack
        if inside:
            assert rec["exit_code"][p] == 9, p          # truncated inside the box
        elif outside:
            assert rec["exit_code"][p] == 1, p          # missed the open face


def test_forward_direct_excitation_ends_at_wall_reflections():
    """Without excitation scattering a path that has not emitted ends at its
    first wall reflection: in an empty box every reflection is such an end."""
    sc = workloads.dark_box_scene(width=8, height=8, n_bins=11, wall_rho=0.7)
    run = workloads.make_run(1 << 14, seed=4, excitation_scatter=False)
    t = oracle.tallies_dict(oracle.render(sc, run)["tallies"])
    assert t["wall_reflect"] > 0
    assert t["exit_excscat"] == t["wall_reflect"]
    full = oracle.tallies_dict(oracle.render(sc, dict(run, excitation_scatter=True))["tallies"])
    assert full["exit_excscat"] == 0 and full["wall_reflect"] > t["wall_reflect"]
