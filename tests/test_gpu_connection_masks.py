"""The host's precomputed pinhole-connection geometry (eqs. 3-6), checked by
brute force in fp64.

For a box scene with a pinhole camera the library marks the spheres whose
every point passes a camera connection's geometric tests (in the image, out
through the open face, clear of the light quad) and, per sphere, the spheres a
segment from it to the eye can meet; the kernels then skip those tests and the
other spheres' chords for such connections.  Both claims are checked here on
points sampled throughout each sphere (its surface included): every segment
from a marked sphere passes every test, and no segment from sphere s meets a
sphere outside s's occluder mask.  A scene built to defeat the shortcuts
(spheres cut by the image's edges, two spheres in line with the eye) shows the
marks are not vacuous."""
from __future__ import annotations

import copy

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _sphere_points(c, r, n, rng):
    """n points inside the ball and n on its surface."""
    d = rng.normal(size=(2 * n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = np.concatenate([r * rng.random(n) ** (1.0 / 3.0), np.full(n, r)])
    return np.asarray(c, float) + d * rad[:, None]


def _camera(sensor):
    eye = np.asarray(sensor["eye"], float)
    f = np.asarray(sensor["look"], float) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(sensor["up"], float))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    ty = np.tan(np.radians(sensor["fov_y_deg"]) / 2)
    tx = ty * sensor["width"] / sensor["height"]
    return eye, f, r, u, tx, ty


def _passes(scene, x):
    """The connection's geometric tests for points x (rows), in fp64."""
    geo, sen, li = scene["geometry"], scene["sensor"], scene["light"]
    eye, f, r, u, tx, ty = _camera(sen)
    v = x - eye
    zc = v @ f
    xi = (v @ r) / (zc * tx)
    yi = (v @ u) / (zc * ty)
    ok = (zc > 0) & (np.abs(xi) < 1) & (np.abs(yi) < 1)
    lo, hi = np.asarray(geo["lo"], float), np.asarray(geo["hi"], float)
    ax, side = geo["open_face"] >> 1, geo["open_face"] & 1
    plane = hi[ax] if side else lo[ax]
    t = (plane - x[:, ax]) / (eye[ax] - x[:, ax])
    q = x + t[:, None] * (eye - x)
    others = [a for a in range(3) if a != ax]
    ok &= (t > 0) & (t < 1)
    for a in others:
        ok &= (q[:, a] >= lo[a]) & (q[:, a] <= hi[a])
    c0 = np.asarray(li["corner"], float)
    lu, lv = np.asarray(li["u"], float), np.asarray(li["v"], float)
    n = np.cross(lu, lv)
    dn = (eye - x) @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        tl = ((c0 - x) @ n) / dn
    ql = x + tl[:, None] * (eye - x) - c0
    a = (ql @ lu) / (lu @ lu)
    b = (ql @ lv) / (lv @ lv)
    blocked = (dn != 0) & (tl > 0) & (tl < 1) & (a >= 0) & (a <= 1) & (b >= 0) & (b <= 1)
    return ok & ~blocked


def _meets(x, eye, c, r):
    """Whether the segments x -> eye meet the ball (c, r)."""
    d = eye - x
    t = np.clip(((np.asarray(c, float) - x) * d).sum(1) / (d * d).sum(1), 0.0, 1.0)
    p = x + t[:, None] * d
    return np.linalg.norm(p - np.asarray(c, float), axis=1) <= r


def _check(scene, seed=7, n=4000):
    import paper_1706_03024_amd as fpt
    sc = fpt.Scene(scene)
    clear, occl = sc.connection_masks()
    sc.close()
    spheres = scene["geometry"]["spheres"]
    eye = np.asarray(scene["sensor"]["eye"], float)
    rng = np.random.default_rng(seed)
    for s, sp in enumerate(spheres):
        x = _sphere_points(sp["center"], sp["radius"], n, rng)
        assert occl[s] >> s & 1, (s, occl)
        if clear >> s & 1:
            good = _passes(scene, x)
            assert good.all(), (s, int((~good).sum()))
        for t, tp in enumerate(spheres):
            if t != s and not (occl[s] >> t & 1):
                hit = _meets(x, eye, tp["center"], tp["radius"])
                assert not hit.any(), (s, t, int(hit.sum()))
    return clear, occl


@pytest.mark.parametrize("name", ["cornell", "large", "glossy", "validation", "maximal"])
def test_masks_hold_on_the_workloads(name):
    scene = {"cornell": lambda: workloads.cornell_scene(128, 128),
             "large": lambda: workloads.large_scene(512, 512),
             "glossy": lambda: workloads.glossy_cornell_scene(64, 64),
             "validation": lambda: workloads.validation_scene(),
             "maximal": lambda: workloads.maximal_scene()}[name]()
    clear, occl = _check(scene)
    if name in ("cornell", "large"):
        # every sphere of the benchmark scenes takes the shortcuts
        n = len(scene["geometry"]["spheres"])
        assert clear == (1 << n) - 1 and all(o == 1 << s for s, o in enumerate(occl)), (clear, occl)


def test_masks_are_not_vacuous():
    """Spheres cut by the image's right and top edges are not clear (some of
    their points fail the image test), a sphere fully inside is; a sphere
    behind another, in line with the eye, has it in its occluder mask (some of
    its segments meet it), while the front one does not have the back one (it
    lies entirely farther from the eye)."""
    s = copy.deepcopy(workloads.cornell_scene(64, 64))
    geo = s["geometry"]
    med = geo["spheres"][0]["medium"]
    geo["spheres"] = [
        {"center": [0.0, -0.5, 0.0], "radius": 0.15, "medium": med},    # clear, in front
        {"center": [0.0, -0.5, -0.6], "radius": 0.15, "medium": med},   # behind it, in line with the eye
        {"center": [0.9, 0.0, -0.9], "radius": 0.08, "medium": med},    # cut by the image's right edge
        {"center": [0.0, 0.72, 0.0], "radius": 0.1, "medium": med},     # cut by the image's top edge
    ]
    s["sensor"] = dict(s["sensor"], fov_y_deg=24.0)
    clear, occl = _check(s)
    rng = np.random.default_rng(3)
    for k in (2, 3):
        sp = geo["spheres"][k]
        x = _sphere_points(sp["center"], sp["radius"], 4000, rng)
        assert not _passes(s, x).all(), k          # the scene really cuts it
        assert not (clear >> k & 1), (k, clear)
    assert clear & 1, clear
    eye = np.asarray(s["sensor"]["eye"], float)
    x1 = _sphere_points(geo["spheres"][1]["center"], 0.15, 4000, rng)
    assert _meets(x1, eye, geo["spheres"][0]["center"], 0.15).any()
    assert occl[1] & 1 and not (occl[0] >> 1 & 1), occl
