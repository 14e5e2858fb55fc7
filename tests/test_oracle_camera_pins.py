"""Pins of the oracle's pinhole splat (eqs. 3-6: geometry term 1/r^2, visibility,
transmittance; importance W_e normalised so that a uniform radiance reads as
itself) against radiance integrals evaluated by quadrature."""
from __future__ import annotations

import math

import numpy as np

import closed_forms as cf
import oracle
import workloads
from stats import check_z

B = 64  # batches for batch-mean standard errors


def _camera(scene):
    se = scene["sensor"]
    return cf.Pinhole(se["eye"], se["look"], se["up"], se["fov_y_deg"], se["width"],
                      se["height"])


def _classify(scene, cam, px, py, sub=3, corners=False):
    """What the sub-pixel rays of pixel (px, py) see first: returns a list of
    (kind, point, direction) with kind in {'light', 'sphere', 'wallF', 'none'}.
    Rays go through the Gauss points of the pixel, or with corners=True through
    its four corners and centre (the image of a convex region is convex, so a
    pixel whose corners all see it lies entirely inside it)."""
    geo = scene["geometry"]
    lo, hi = np.array(geo["lo"]), np.array(geo["hi"])
    li = scene["light"]
    corner, u, v = (np.array(li[k], float) for k in ("corner", "u", "v"))
    g, _ = np.polynomial.legendre.leggauss(sub)
    pts = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (0.5, 0.5)] if corners else \
        [(a, b) for a in 0.5 * (g + 1) for b in 0.5 * (g + 1)]
    out = []
    for a, b in pts:
        if True:
            d = cam.ray(px + a, py + b)
            # enter through the open face z = hi
            t_in = (hi[2] - cam.eye[2]) / d[2]
            p = cam.eye + t_in * d
            if not (lo[0] <= p[0] <= hi[0] and lo[1] <= p[1] <= hi[1]):
                out.append(("none", None, d))
                continue
            t_wall = cf.ray_box_exit(p, d, lo, hi)
            t_light = cf.ray_plane_rect(p, d, corner, u, v)
            t_sph = np.inf
            for sp in geo["spheres"]:
                t0, _ = cf.ray_sphere(p, d, np.array(sp["center"]), sp["radius"])
                if np.isfinite(t0) and t0 > 0:
                    t_sph = min(t_sph, t0)
            tm = min(t_wall, t_light, t_sph)
            if tm == t_light:
                out.append(("light", p + tm * d, d))
            elif tm == t_sph:
                out.append(("sphere", p + tm * d, d))
            else:
                q = p + tm * d
                face = int(np.argmin(np.abs(np.concatenate([q - lo, hi - q]))))
                face = (face % 3) * 2 + (1 if face >= 3 else 0)
                out.append((f"wall{face}", q, d))
    return out


def _batches(scene, n, seed, **kw):
    run = workloads.make_run(n, seed=seed, parity_batches=B, **kw)
    return oracle.render(scene, run)["film"]


def test_direct_view_of_light_reads_its_radiance():
    """A Lambertian quad of power P and area A has radiance P/(pi A); pixels
    entirely covered by it read that value in the line's bin."""
    s = workloads.dark_box_scene(width=64, height=64, lines=[(550, 1.0)])
    cam = _camera(s)
    film = _batches(s, 1 << 17, seed=1)
    L = 1.0 / (math.pi * 0.25)
    z = []
    covered = 0
    for py in range(12):
        for px in range(64):
            kinds = {k for k, _, _ in _classify(s, cam, px, py, corners=True)}
            if kinds == {"light"}:
                covered += 1
                vals = film[:, 0, py, px, 50]
                z.append((vals.mean() - L) / (vals.std(ddof=1) / math.sqrt(B)))
                assert film[:, :, py, px, :50].sum() == 0.0
    assert covered >= 4
    check_z(z, "direct light radiance", dof=B - 1)


def test_first_bounce_wall_radiance():
    """A Lambertian back wall of reflectance rho lit only by the quad has
    radiance rho/pi * E(x), E the quad's irradiance (other walls black)."""
    W = 24
    s = workloads.dark_box_scene(width=W, height=W, lines=[(550, 1.0)])
    rho = 0.5
    s["geometry"]["walls"][4] = workloads.pwl((300, rho), (800, rho))
    cam = _camera(s)
    film = _batches(s, 1 << 19, seed=2)
    li = s["light"]
    corner, u, v = (np.array(li[k], float) for k in ("corner", "u", "v"))
    Le = 1.0 / (math.pi * 0.25)
    z = []
    for py in range(0, W, 2):
        for px in range(0, W, 2):
            if any(k != "wall4" for k, _, _ in _classify(s, cam, px, py, corners=True)):
                continue
            cls = _classify(s, cam, px, py, sub=3)
            g, wg = np.polynomial.legendre.leggauss(3)
            wts = np.outer(wg, wg).ravel() / 4.0
            Ls = [rho / math.pi * cf.quad_irradiance(q, np.array([0, 0, 1.0]), corner, u, v, Le,
                                                      n=24) for _, q, _ in cls]
            expect = float(np.dot(wts, Ls))
            vals = film[:, 0, py, px, 50]
            z.append((vals.mean() - expect) / (vals.std(ddof=1) / math.sqrt(B)))
    assert len(z) >= 20
    check_z(z, "first-bounce wall radiance", dof=B - 1)


def test_single_scatter_radiance_of_a_sphere():
    """With one allowed scatter and black walls, pixels that see the sphere read
    the single-scattering radiance: int T sigma_s/(4 pi) (int L_e T cos/r^2 dA) dt."""
    W = 24
    sig_s, sig_a = 1.5, 0.5
    med = {"sigma_s": sig_s, "sigma_a_bg": sig_a, "dyes": []}
    s = workloads.dark_box_scene(sphere_medium=med, width=W, height=W, lines=[(550, 1.0)])
    cam = _camera(s)
    film = _batches(s, 1 << 20, seed=3, max_scatter=1)
    li = s["light"]
    corner, u, v = (np.array(li[k], float) for k in ("corner", "u", "v"))
    sp = s["geometry"]["spheres"][0]
    c, r = np.array(sp["center"]), sp["radius"]
    Le = 1.0 / (math.pi * 0.25)
    z = []
    for py in range(W):
        for px in range(W):
            if any(k != "sphere" for k, _, _ in _classify(s, cam, px, py, corners=True)):
                continue
            cls = _classify(s, cam, px, py, sub=2)
            g, wg = np.polynomial.legendre.leggauss(2)
            wts = np.outer(wg, wg).ravel() / 4.0
            Ls = [cf.single_scatter_radiance(cam.eye, d, c, r, sig_s, sig_s + sig_a, corner, u,
                                             v, Le, n_line=12, n_quad=16) for _, _, d in cls]
            expect = float(np.dot(wts, Ls))
            vals = film[:, 0, py, px, 50]
            z.append((vals.mean() - expect) / (vals.std(ddof=1) / math.sqrt(B)))
    assert len(z) >= 6
    check_z(z, "single-scatter sphere radiance", dof=B - 1)
