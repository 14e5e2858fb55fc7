"""Seeded synthetic workloads for the fluorescent spectral path tracer.

This module only *describes* inputs: scene, medium, dye, light and sensor
parameters as plain dictionaries, plus the seeded generator for the batched
instance table.  It holds none of the transport arithmetic; both the GPU
library binding and the CPU oracle marshal these dictionaries into their own
C structures.

Scene dictionary schema (units: nm, mm, 1/mm, 1/(M cm), uM):

    grid      {"n_bins": N, "lo_nm": 300, "hi_nm": 800}
              N points lambda_k = lo + k*(hi-lo)/(N-1); bin k is centred on lambda_k.
    absorptivity_base  "decadic" (sigma_a = ln10*eps*c*a_hat) or "natural" (eps*c*a_hat)
    dyes      [{"absorption": spectrum, "emission": spectrum, "epsilon": e, "qy": q}]
    media     [{"sigma_s": s, "sigma_a_bg": a, "dyes": [[dye_index, conc_uM], ...]}]
    geometry  {"kind": "slab", "z0", "z1", "medium"} | {"kind": "halfspace", "z0", "medium"}
              | {"kind": "sphere", "center", "radius", "medium"} | {"kind": "infinite", "medium"}
              | {"kind": "box", "lo", "hi", "open_face", "walls": [spectrum|None]*6,
                 "spheres": [{"center", "radius", "medium"}]}
              Box faces: 0 x=lo, 1 x=hi, 2 y=lo, 3 y=hi, 4 z=lo, 5 z=hi.
    light     {"kind": "beam", "pos", "dir", "lines"} | {"kind": "point", "pos", "lines"}
              | {"kind": "quad", "corner", "u", "v", "lines"};  lines = [[nm, power], ...]
    sensor    {"kind": "escape"} | {"kind": "pinhole", "eye", "look", "up", "fov_y_deg",
                                     "width", "height"}

    spectrum  {"gauss": [[mean_nm, sd_nm, weight], ...]} | {"pwl": [[nm, value], ...]}

Run dictionary: {"seed", "instance", "path_begin", "path_count", "total_paths",
"max_scatter", "max_emissions", "fluorescence_only", "excitation_scatter",
"parity_batches", "splat_rr"}.
"""
from __future__ import annotations

import copy
import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))

UNLIMITED_EMISSIONS = 0xFFFFFFFF


def gauss(*terms):
    """Spectrum as a Gaussian mixture: terms are (mean_nm, sd_nm, weight)."""
    return {"gauss": [list(map(float, t)) for t in terms]}


def pwl(*knots):
    """Spectrum as a piecewise-linear curve through (nm, value) knots."""
    return {"pwl": [list(map(float, k)) for k in knots]}


def make_run(path_count, seed=0, instance=0, path_begin=0, total_paths=None,
             max_scatter=10000, max_emissions=1, fluorescence_only=False,
             excitation_scatter=True, parity_batches=1, splat_rr=0.0):
    return {
        "seed": int(seed), "instance": int(instance),
        "path_begin": int(path_begin), "path_count": int(path_count),
        "total_paths": int(total_paths if total_paths is not None else path_count),
        "max_scatter": int(max_scatter), "max_emissions": int(max_emissions),
        "fluorescence_only": bool(fluorescence_only),
        "excitation_scatter": bool(excitation_scatter),
        "parity_batches": int(parity_batches), "splat_rr": float(splat_rr),
    }


def grid(n_bins=101, lo=300.0, hi=800.0):
    return {"n_bins": int(n_bins), "lo_nm": float(lo), "hi_nm": float(hi)}


# --------------------------------------------------------------------------
# Plain slab: 1 mm, sigma_s 10/mm, one Gaussian dye, 490 nm beam, 2^16 paths.
# --------------------------------------------------------------------------
def slab_scene(sigma_s=10.0, sigma_a_bg=0.01, conc_uM=10.0, qy=0.9, epsilon=7e4,
               lambda_x=490.0, thickness=1.0, n_bins=101):
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": [{"absorption": gauss((490, 20, 1)), "emission": gauss((520, 25, 1)),
                  "epsilon": epsilon, "qy": qy}],
        "media": [{"sigma_s": sigma_s, "sigma_a_bg": sigma_a_bg,
                   "dyes": [[0, conc_uM]] if conc_uM > 0 else []}],
        "geometry": {"kind": "slab", "z0": 0.0, "z1": float(thickness), "medium": 0},
        "light": {"kind": "beam", "pos": [0.0, 0.0, 0.0], "dir": [0.0, 0.0, 1.0],
                  "lines": [[lambda_x, 1.0]]},
        "sensor": {"kind": "escape"},
    }


def slab_config():
    return slab_scene(), make_run(1 << 16, seed=0)


# --------------------------------------------------------------------------
# Cornell-style box: three dye spheres, piecewise-linear walls, quad light.
# --------------------------------------------------------------------------
RED_WALL = pwl((300, .05), (580, .05), (620, .70), (800, .75))
GREEN_WALL = pwl((300, .05), (480, .10), (530, .60), (580, .10), (800, .05))
WHITE_WALL = pwl((300, .60), (400, .75), (800, .80))


def _box_walls():
    # faces: 0 x=-1 (red), 1 x=+1 (green), 2 floor, 3 ceiling, 4 back, 5 open front
    return [RED_WALL, GREEN_WALL, WHITE_WALL, WHITE_WALL, WHITE_WALL, None]


def _quad_light(lines):
    return {"kind": "quad", "corner": [-0.25, 0.999, -0.25], "u": [0.5, 0.0, 0.0],
            "v": [0.0, 0.0, 0.5], "lines": [[float(nm), float(p)] for nm, p in lines]}


def _pinhole(width, height):
    return {"kind": "pinhole", "eye": [0.0, 0.0, 3.4], "look": [0.0, 0.0, 0.0],
            "up": [0.0, 1.0, 0.0], "fov_y_deg": 40.0, "width": int(width),
            "height": int(height)}


CORNELL_DYES = [  # (abs mean, abs sd, em mean, em sd, epsilon, qy, conc uM, sigma_s)
    (450, 20, 475, 25, 3e4, 0.50, 50.0, 50.0),
    (550, 20, 580, 25, 7e4, 0.80, 10.0, 100.0),
    (650, 20, 690, 30, 1e5, 0.95, 1.0, 200.0),
]
# Sphere centres; lifted 0.01 mm above the floor so no medium touches a wall.
CORNELL_SPHERES = [(-0.5, -0.79, -0.2), (0.0, -0.79, 0.2), (0.5, -0.79, -0.2)]


def cornell_scene(width=128, height=128, conc_scale=(1.0, 1.0, 1.0), n_bins=101):
    dyes, media, spheres = [], [], []
    for i, (am, asd, em, esd, eps, qy, c, ss) in enumerate(CORNELL_DYES):
        dyes.append({"absorption": gauss((am, asd, 1)), "emission": gauss((em, esd, 1)),
                     "epsilon": eps, "qy": qy})
        media.append({"sigma_s": ss, "sigma_a_bg": 0.01, "dyes": [[i, c * conc_scale[i]]]})
        spheres.append({"center": list(CORNELL_SPHERES[i]), "radius": 0.2, "medium": i})
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dyes,
        "media": media,
        "geometry": {"kind": "box", "lo": [-1.0, -1.0, -1.0], "hi": [1.0, 1.0, 1.0],
                     "open_face": 5, "walls": _box_walls(), "spheres": spheres},
        "light": _quad_light([(450, 1.0), (550, 1.0), (650, 1.0)]),
        "sensor": _pinhole(width, height),
    }


def glossy_cornell_scene(width=128, height=128, back=30.0, floor=8.0, n_bins=101):
    """The Cornell scene with glossy walls (the paper's glossy Cornell box,
    sec. 5): back wall and floor reflect with normalised modified-Phong lobes
    of exponent `back` and `floor` about the mirror direction."""
    s = cornell_scene(width, height, n_bins=n_bins)
    s["geometry"]["wall_gloss"] = [0.0, 0.0, float(floor), 0.0, float(back), 0.0]
    return s


def cornell_config():
    """128x128 pinhole, 64 spp (2^20 light paths), 101 bins."""
    return cornell_scene(), make_run(128 * 128 * 64, seed=0)


def camera_config(spp=8):
    """The Cornell scene rendered camera-side: 128x128 pixels x 101 emission
    bins x spp samples (13.2M paths at 8 samples)."""
    scene = cornell_scene()
    return scene, make_run(spp * 128 * 128 * 101, seed=0)


# --------------------------------------------------------------------------
# Large highly scattering scene: five bimodal dyes, sigma_s up to 1000/mm.
# --------------------------------------------------------------------------
LARGE_DYES = [  # abs (m1,s1),(m2,s2); em (m1,s1),(m2,s2); eps; qy; c; sigma_s
    ((400, 15), (350, 20), (440, 20), (470, 25), 5e4, 0.6, 20.0, 200.0),
    ((490, 18), (460, 20), (520, 20), (550, 25), 7e4, 0.9, 10.0, 500.0),
    ((550, 20), (515, 20), (580, 20), (620, 25), 9e4, 0.7, 5.0, 1000.0),
    ((600, 20), (565, 20), (640, 22), (680, 25), 1e5, 0.5, 2.0, 1000.0),
    ((650, 20), (610, 20), (700, 25), (740, 30), 1e5, 0.3, 1.0, 800.0),
]


def large_scene(width=512, height=512, n_bins=301):
    dyes, media, spheres = [], [], []
    xs = [-0.72, -0.36, 0.0, 0.36, 0.72]
    for i, (a1, a2, e1, e2, eps, qy, c, ss) in enumerate(LARGE_DYES):
        dyes.append({"absorption": gauss((a1[0], a1[1], 1.0), (a2[0], a2[1], 0.3)),
                     "emission": gauss((e1[0], e1[1], 1.0), (e2[0], e2[1], 0.4)),
                     "epsilon": eps, "qy": qy})
        media.append({"sigma_s": ss, "sigma_a_bg": 0.01, "dyes": [[i, c]]})
        spheres.append({"center": [xs[i], -0.82, 0.2 if i % 2 == 0 else -0.2],
                        "radius": 0.17, "medium": i})
    lines = [(d[0][0], 1.0) for d in LARGE_DYES]
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dyes,
        "media": media,
        "geometry": {"kind": "box", "lo": [-1.0, -1.0, -1.0], "hi": [1.0, 1.0, 1.0],
                     "open_face": 5, "walls": _box_walls(), "spheres": spheres},
        "light": _quad_light(lines),
        "sensor": _pinhole(width, height),
    }


def large_config():
    """512x512 pinhole, 1024 spp (2^28 light paths), 301 bins, scatter cap 1e4."""
    return large_scene(), make_run(512 * 512 * 1024, seed=0, max_scatter=10000)


# --------------------------------------------------------------------------
# Adjoint workload: the Cornell geometry and dyes at 256x256, 256 spp.
# --------------------------------------------------------------------------
ADJOINT_HIDDEN_CONC_SCALE = (1.5, 0.7, 1.3)


def adjoint_config(width=256, height=256, spp=256):
    scene = cornell_scene(width, height)
    target = cornell_scene(width, height, conc_scale=ADJOINT_HIDDEN_CONC_SCALE)
    n = width * height * spp
    return scene, make_run(n, seed=0), target, make_run(n, seed=1)


# --------------------------------------------------------------------------
# Batched instances: slabs and spheres with 1-3 random dyes each.
# --------------------------------------------------------------------------
BATCH_JSON = os.path.join(_HERE, "batch_instances.json")


def generate_batch_instances(n=1024, seed=2024):
    """Draw the batched instance table with numpy's PCG64 (parameters only)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))

    def logu(lo, hi):
        return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))

    out = []
    for i in range(n):
        geom = "slab" if rng.integers(0, 2) == 0 else "sphere"
        nd = int(rng.integers(1, 4))
        dyes = []
        for _ in range(nd):
            am = float(rng.uniform(350, 650))
            asd = float(rng.uniform(15, 30))
            stokes = float(rng.uniform(20, 40))
            esd = float(rng.uniform(20, 35))
            eps = logu(3e4, 1e5)
            conc = logu(0.1, 100.0)
            qy = float(rng.uniform(0.3, 1.0))
            dyes.append({"abs_mean": am, "abs_sd": asd, "em_mean": am + stokes, "em_sd": esd,
                         "epsilon": eps, "conc_uM": conc, "qy": qy})
        sigma_s = logu(1.0, 500.0)
        lx = float(rng.uniform(350, 650))
        lx = 5.0 * round(lx / 5.0)
        log2_paths = int(rng.integers(12, 19))
        out.append({"geometry": geom, "dyes": dyes, "sigma_s": sigma_s, "lambda_x": lx,
                    "paths": 1 << log2_paths, "instance": i})
    return out


def load_batch_instances():
    with open(BATCH_JSON) as f:
        return json.load(f)


def batch_instance_scene(inst, n_bins=101):
    dyes = [{"absorption": gauss((d["abs_mean"], d["abs_sd"], 1.0)),
             "emission": gauss((d["em_mean"], d["em_sd"], 1.0)),
             "epsilon": d["epsilon"], "qy": d["qy"]} for d in inst["dyes"]]
    media = [{"sigma_s": inst["sigma_s"], "sigma_a_bg": 0.01,
              "dyes": [[j, d["conc_uM"]] for j, d in enumerate(inst["dyes"])]}]
    if inst["geometry"] == "slab":
        geom = {"kind": "slab", "z0": 0.0, "z1": 1.0, "medium": 0}
        light_pos = [0.0, 0.0, 0.0]
    else:
        geom = {"kind": "sphere", "center": [0.0, 0.0, 0.5], "radius": 0.5, "medium": 0}
        light_pos = [0.0, 0.0, 0.0]  # south pole, beam along the diameter
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dyes,
        "media": media,
        "geometry": geom,
        "light": {"kind": "beam", "pos": light_pos, "dir": [0.0, 0.0, 1.0],
                  "lines": [[inst["lambda_x"], 1.0]]},
        "sensor": {"kind": "escape"},
    }


def batch_config(instances=None):
    """Scenes and runs for the batched workload (instance key = instance id, seed 0)."""
    if instances is None:
        instances = load_batch_instances()
    scenes = [batch_instance_scene(inst) for inst in instances]
    runs = [make_run(inst["paths"], seed=0, instance=inst["instance"]) for inst in instances]
    return scenes, runs


# --------------------------------------------------------------------------
# The paper's experiments as batched sweeps (sec. 5: one dye, its excitation
# varied across the spectrum, and its concentration varied at fixed
# illumination).  Each instance is a 1 mm slab of the dye's solution lit by a
# normal beam and read by escape tallies; the instance key is its index.
# --------------------------------------------------------------------------
SWEEP_DYE = {"abs": (490.0, 20.0), "em": (520.0, 25.0), "epsilon": 7e4, "qy": 0.9}


def sweep_slab(lambda_x, conc_uM, sigma_s=0.0, sigma_a_bg=0.01, d=1.0, n_bins=101):
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, sigma_s, sigma_a_bg,
                       dyes=[conc_uM], light=_beam(lambda_x), n_bins=n_bins,
                       absorption=gauss((*SWEEP_DYE["abs"], 1.0)),
                       emission=gauss((*SWEEP_DYE["em"], 1.0)),
                       epsilon=SWEEP_DYE["epsilon"], qy=SWEEP_DYE["qy"])


def excitation_scan(lambdas=None, conc_uM=10.0, sigma_s=0.0, paths=1 << 18, seed=0):
    """Excitation wavelengths 300-700 nm in 5 nm steps (81 instances)."""
    if lambdas is None:
        lambdas = [300.0 + 5.0 * i for i in range(81)]
    scenes = [sweep_slab(lx, conc_uM, sigma_s) for lx in lambdas]
    runs = [make_run(paths, seed=seed, instance=i) for i in range(len(scenes))]
    return scenes, runs


def concentration_sweep(concs=None, lambda_x=490.0, sigma_s=0.0, paths=1 << 18, seed=0):
    """Concentrations 0.1-1000 uM, four per decade (17 instances)."""
    if concs is None:
        concs = [10.0 ** (-1.0 + 0.25 * i) for i in range(17)]
    scenes = [sweep_slab(lambda_x, c, sigma_s) for c in concs]
    runs = [make_run(paths, seed=seed, instance=i) for i in range(len(scenes))]
    return scenes, runs


# --------------------------------------------------------------------------
# Closed-form test scenes.
# --------------------------------------------------------------------------
def _one_medium(geometry, sigma_s, sigma_a_bg, dyes=(), light=None, n_bins=101,
                absorption=None, emission=None, epsilon=7e4, qy=0.9):
    dye_list = []
    media_dyes = []
    for j, conc in enumerate(dyes):
        dye_list.append({"absorption": absorption or gauss((490, 20, 1)),
                         "emission": emission or gauss((520, 25, 1)),
                         "epsilon": epsilon, "qy": qy})
        media_dyes.append([j, conc])
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dye_list,
        "media": [{"sigma_s": sigma_s, "sigma_a_bg": sigma_a_bg, "dyes": media_dyes}],
        "geometry": geometry,
        "light": light,
        "sensor": {"kind": "escape"},
    }


def _beam(nm=490.0, z0=0.0):
    return {"kind": "beam", "pos": [0.0, 0.0, z0], "dir": [0.0, 0.0, 1.0], "lines": [[nm, 1.0]]}


def t1_beer_lambert(d=1.0, sigma_s=0.5, sigma_a=0.5):
    """Absorbing and scattering slab, no dye: ballistic transmission."""
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, sigma_s, sigma_a,
                       light=_beam())


def t2_infinite(albedo, sigma_t=1.0):
    """Infinite medium, isotropic point source, no dye."""
    return _one_medium({"kind": "infinite", "medium": 0}, albedo * sigma_t,
                       (1 - albedo) * sigma_t,
                       light={"kind": "point", "pos": [0.0, 0.0, 0.0], "lines": [[490.0, 1.0]]})


def t3_conservative_slab(tau=10.0, d=1.0):
    """Non-absorbing slab: every path escapes or is capped."""
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, tau / d, 0.0,
                       light=_beam())


def t4_infinite_dye(qy=0.7, sigma_s=0.0, conc_uM=10.0):
    """Infinite medium with one dye and no background absorber.

    A broad absorption band keeps sigma_a > 0 at every emission wavelength, so
    every path ends in a non-radiative decay (or, with K=1, a second absorption).
    """
    return _one_medium({"kind": "infinite", "medium": 0}, sigma_s, 0.0, dyes=[conc_uM],
                       absorption=gauss((500, 120, 1)), emission=gauss((560, 30, 1)),
                       qy=qy,
                       light={"kind": "point", "pos": [0.0, 0.0, 0.0], "lines": [[490.0, 1.0]]})


def t5_thin_dye_slab(conc_uM=0.1, sigma_s=0.1):
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": 1.0, "medium": 0}, sigma_s, 0.0,
                       dyes=[conc_uM], light=_beam())


def t6_dye_slab(lambda_x=490.0, conc_uM=10.0, sigma_a_bg=0.05, d=1.0, qy=0.9):
    """Non-scattering dye slab: fluorescent escape film has a 1-D quadrature form."""
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, 0.0, sigma_a_bg,
                       dyes=[conc_uM], qy=qy, light=_beam(lambda_x))


def t7_single_scatter(tau=0.05, d=1.0):
    return _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, tau / d, 0.0,
                       light=_beam())


def t8_halfspace(albedo, sigma_t=1.0):
    return _one_medium({"kind": "halfspace", "z0": 0.0, "medium": 0}, albedo * sigma_t,
                       (1 - albedo) * sigma_t, light=_beam())


def t9_dielectric_slab_beam(ior, theta_deg, sigma_a=0.5, d=1.0, sigma_s=0.0):
    """Slab of refractive index `ior` (vacuum outside) hit by a beam at
    theta_deg from the normal."""
    th = math.radians(theta_deg)
    light = {"kind": "beam", "pos": [0.0, 0.0, 0.0], "dir": [math.sin(th), 0.0, math.cos(th)],
             "lines": [[490.0, 1.0]]}
    s = _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, sigma_s, sigma_a, light=light)
    s["media"][0]["ior"] = float(ior)
    return s


def t10_dielectric_slab_point(ior, sigma_a=0.3, d=1.0, zs=0.3, sigma_s=0.0):
    """Isotropic point source at height zs inside a refractive slab [0, d]."""
    light = {"kind": "point", "pos": [0.0, 0.0, zs], "lines": [[490.0, 1.0]]}
    s = _one_medium({"kind": "slab", "z0": 0.0, "z1": d, "medium": 0}, sigma_s, sigma_a, light=light)
    s["media"][0]["ior"] = float(ior)
    return s


def t11_dielectric_sphere_point(ior, sigma_a=0.5, radius=1.0, offset=0.8, sigma_s=0.0):
    """Isotropic point source at `offset` from the centre of a refractive sphere."""
    light = {"kind": "point", "pos": [0.0, offset, radius], "lines": [[490.0, 1.0]]}
    s = _one_medium({"kind": "sphere", "center": [0.0, 0.0, radius], "radius": radius, "medium": 0},
                    sigma_s, sigma_a, light=light)
    s["media"][0]["ior"] = float(ior)
    return s


def sphere_scene(radius=0.5, sigma_s=20.0, sigma_a_bg=0.01, conc_uM=10.0, lambda_x=490.0):
    s = slab_scene(sigma_s=sigma_s, sigma_a_bg=sigma_a_bg, conc_uM=conc_uM,
                   lambda_x=lambda_x)
    s["geometry"] = {"kind": "sphere", "center": [0.0, 0.0, radius], "radius": radius,
                     "medium": 0}
    return s


def dark_box_scene(sphere_medium=None, width=32, height=32, n_bins=101, lines=None,
                   wall_rho=0.0):
    """Box with uniform (default black) walls, for camera closed-form checks."""
    walls = [pwl((300, wall_rho), (800, wall_rho))] * 5 + [None]
    spheres = []
    media = []
    dyes = []
    if sphere_medium is not None:
        media.append(sphere_medium)
        spheres.append({"center": [0.0, -0.3, 0.0], "radius": 0.3, "medium": 0})
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dyes,
        "media": media,
        "geometry": {"kind": "box", "lo": [-1.0, -1.0, -1.0], "hi": [1.0, 1.0, 1.0],
                     "open_face": 5, "walls": walls, "spheres": spheres},
        "light": _quad_light(lines or [(550, 1.0)]),
        "sensor": _pinhole(width, height),
    }


def validation_scene(lambda_x=550.0, conc_uM=1.0, sigma_s=20.0, width=32, n_bins=101):
    """The paper's spectral validation (sec. 6, Figs. 6-7) as a synthetic scene:
    one sphere of a single Gaussian dye (absorption 550/20 nm, emission 580/25 nm,
    epsilon 7e4, QY 0.8) in a box with black walls, lit at one excitation line,
    seen by a pinhole; weak dye (1 uM) so reabsorption barely reshapes the
    escaping fluorescence."""
    med = {"sigma_s": sigma_s, "sigma_a_bg": 0.01, "dyes": [[0, conc_uM]]}
    s = dark_box_scene(sphere_medium=med, width=width, height=width, n_bins=n_bins,
                       lines=[(lambda_x, 1.0)])
    s["dyes"] = [{"absorption": gauss((550.0, 20.0, 1.0)), "emission": gauss((580.0, 25.0, 1.0)),
                  "epsilon": 7e4, "qy": 0.8}]
    return s


def maximal_scene(n_bins=101, width=16):
    """The box at every descriptor maximum the ABI allows: 8 spheres, each of
    its own medium; 8 dyes, 4 in every medium; 8 light lines; a 16-term
    absorption spectrum.  Spheres of radius 0.22 sit at (+-0.5, +-0.5, +-0.5);
    scattering 4-32/mm, concentrations 2-16 uM."""
    dyes = []
    for i in range(8):
        a_mean, e_mean = 380.0 + 45.0 * i, 420.0 + 45.0 * i
        absorption = gauss((a_mean, 18.0, 1.0), (a_mean - 30.0, 25.0, 0.3))
        if i == 0:   # the most terms a spectrum may have
            absorption = gauss(*[(360.0 + 8.0 * j, 6.0 + j, 1.0 / (1 + j)) for j in range(16)])
        dyes.append({"absorption": absorption, "emission": gauss((e_mean, 22.0, 1.0)),
                     "epsilon": 2e4 + 8e3 * i, "qy": 0.3 + 0.08 * i})
    media, spheres = [], []
    for m in range(8):
        media.append({"sigma_s": 4.0 * (m + 1), "sigma_a_bg": 0.02,
                      "dyes": [[(m + j) % 8, 2.0 * (1 + (m + 3 * j) % 8)] for j in range(4)]})
        c = [0.5 if m & 1 else -0.5, 0.5 if m & 2 else -0.5, 0.5 if m & 4 else -0.5]
        spheres.append({"center": c, "radius": 0.22, "medium": m})
    lines = [(400.0 + 50.0 * i, 1.0 + 0.25 * i) for i in range(8)]
    return {
        "grid": grid(n_bins),
        "absorptivity_base": "decadic",
        "dyes": dyes,
        "media": media,
        "geometry": {"kind": "box", "lo": [-1.0, -1.0, -1.0], "hi": [1.0, 1.0, 1.0],
                     "open_face": 5, "walls": _box_walls(), "spheres": spheres},
        "light": _quad_light(lines),
        "sensor": _pinhole(width, width),
    }


def deepcopy(x):
    return copy.deepcopy(x)


def tabulate(scene, spectrum):
    """The spectrum sampled on the scene's grid, as a tabulated spectrum (the
    form measured spectra take).  Pure sampling of the analytic description."""
    g = scene["grid"]
    n, lo, hi = g["n_bins"], g["lo_nm"], g["hi_nm"]
    lam = [lo + (hi - lo) * k / (n - 1) for k in range(n)]
    if "gauss" in spectrum:
        vals = [sum(w * math.exp(-0.5 * ((x - mu) / sd) ** 2) for mu, sd, w in spectrum["gauss"])
                for x in lam]
    else:
        knots = spectrum["pwl"]
        vals = []
        for x in lam:
            if x <= knots[0][0]:
                vals.append(knots[0][1])
            elif x >= knots[-1][0]:
                vals.append(knots[-1][1])
            else:
                i = next(j for j in range(1, len(knots)) if x <= knots[j][0])
                (x0, y0), (x1, y1) = knots[i - 1], knots[i]
                vals.append(y0 + (x - x0) / (x1 - x0) * (y1 - y0))
    return {"table": vals}


def tabulated_scene(scene):
    """Every dye spectrum and wall reflectance of `scene` as a tabulated spectrum."""
    s = copy.deepcopy(scene)
    for d in s["dyes"]:
        d["absorption"] = tabulate(s, d["absorption"])
        d["emission"] = tabulate(s, d["emission"])
    geo = s["geometry"]
    if geo["kind"] == "box":
        geo["walls"] = [None if w is None else tabulate(s, w) for w in geo["walls"]]
    return s
