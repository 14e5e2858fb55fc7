"""CPU oracle for the fluorescent spectral path tracer -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It wraps ``liboracle.so`` (plain C, fp64,
single-threaded), which shares no code with the GPU library; the scene
dictionaries come from the ``workloads`` module.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_PATH = os.path.join(_HERE, "liboracle.so")
# a sanitizer build of the same source may stand in for it (tests only)
LIB_PATH = os.environ.get("FPT_ORACLE_LIBRARY") or BUILD_PATH

MAX_TERMS, MAX_DYES, MAX_MEDIA, MAX_MEDIUM_DYES, MAX_SPHERES, MAX_LINES = 16, 8, 8, 4, 8, 8

EXIT_NAMES = ["esc_r", "esc_t", "bg", "nonrad", "kcap", "scap", "wall", "light",
              "excscat", "trunc"]
TALLY_NAMES = ["paths", "vertices", "scatters", "dye_abs", "emissions", "wall_reflect",
               "crossings", "splat_hit", "splat_miss", "splat_rr_kill"] + \
              ["exit_" + n for n in EXIT_NAMES]
N_TALLIES = 20


def build(verbose=False):
    """Compile liboracle.so with gcc (-O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
           os.path.join(_HERE, "oracle.c"), "-lm", "-o", BUILD_PATH]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)


class Spectrum(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("x", C.c_double * MAX_TERMS),
                ("y", C.c_double * MAX_TERMS), ("s", C.c_double * MAX_TERMS),
                ("tab", C.c_void_p)]


class Dye(C.Structure):
    _fields_ = [("absorption", Spectrum), ("emission", Spectrum), ("epsilon", C.c_double),
                ("qy", C.c_double)]


class Medium(C.Structure):
    _fields_ = [("sigma_s", C.c_double), ("sigma_a_bg", C.c_double), ("n_dyes", C.c_int32),
                ("dye", C.c_int32 * MAX_MEDIUM_DYES), ("conc", C.c_double * MAX_MEDIUM_DYES),
                ("ior", C.c_double)]


class Sphere(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("radius", C.c_double), ("medium", C.c_int32)]


class Scene(C.Structure):
    _fields_ = [
        ("n_bins", C.c_int32), ("lo_nm", C.c_double), ("hi_nm", C.c_double),
        ("natural_base", C.c_int32),
        ("n_dyes", C.c_int32), ("dyes", Dye * MAX_DYES),
        ("n_media", C.c_int32), ("media", Medium * MAX_MEDIA),
        ("geom", C.c_int32), ("z0", C.c_double), ("z1", C.c_double),
        ("center", C.c_double * 3), ("radius", C.c_double), ("body_medium", C.c_int32),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("open_face", C.c_int32),
        ("walls", Spectrum * 6),
        ("n_spheres", C.c_int32), ("spheres", Sphere * MAX_SPHERES),
        ("light", C.c_int32), ("lpos", C.c_double * 3), ("ldir", C.c_double * 3),
        ("lu", C.c_double * 3), ("lv", C.c_double * 3),
        ("n_lines", C.c_int32), ("line_nm", C.c_double * MAX_LINES),
        ("line_power", C.c_double * MAX_LINES),
        ("sensor", C.c_int32), ("eye", C.c_double * 3), ("look", C.c_double * 3),
        ("up", C.c_double * 3), ("fov_y_deg", C.c_double), ("width", C.c_int32),
        ("height", C.c_int32), ("wall_gloss", C.c_double * 6),
    ]


class Run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("instance", C.c_uint32), ("max_scatter", C.c_uint32),
                ("path_begin", C.c_uint64), ("path_count", C.c_uint64),
                ("total_paths", C.c_uint64), ("max_emissions", C.c_uint32),
                ("fluorescence_only", C.c_int32), ("excitation_scatter", C.c_int32),
                ("parity_batches", C.c_uint32), ("splat_rr", C.c_double),
                ("perturb_eta", C.c_double), ("perturb_pattern", C.c_uint32),
                ("pad_", C.c_uint32)]


class Record(C.Structure):
    _fields_ = [("n_vertices", C.c_uint32), ("n_scatter", C.c_uint32), ("n_emit", C.c_uint32),
                ("exit_code", C.c_uint32), ("lambda_", C.c_int32), ("comp", C.c_int32),
                ("region", C.c_int32), ("pad", C.c_int32), ("pos", C.c_double * 3),
                ("dir", C.c_double * 3), ("splat_sum", C.c_double), ("margin", C.c_double)]


RECORD_DTYPE = np.dtype([("n_vertices", "<u4"), ("n_scatter", "<u4"), ("n_emit", "<u4"),
                         ("exit_code", "<u4"), ("lambda", "<i4"), ("comp", "<i4"),
                         ("region", "<i4"), ("pad", "<i4"), ("pos", "<f8", 3),
                         ("dir", "<f8", 3), ("splat_sum", "<f8"), ("margin", "<f8")])
assert RECORD_DTYPE.itemsize == C.sizeof(Record)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_render.restype = C.c_int32
        L.orc_render.argtypes = [C.POINTER(Scene), C.POINTER(Run), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32]
        L.orc_render_camera.restype = C.c_int32
        L.orc_render_camera.argtypes = [C.POINTER(Scene), C.POINTER(Run), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_uint32]
        L.orc_film_size.restype = C.c_int64
        L.orc_film_size.argtypes = [C.POINTER(Scene), C.c_uint32]
        L.orc_n_params.restype = C.c_int32
        L.orc_n_params.argtypes = [C.POINTER(Scene)]
        L.orc_last_error.restype = C.c_char_p
        L.orc_tables.restype = C.c_int32
        L.orc_tables.argtypes = [C.POINTER(Scene)] + [C.c_void_p] * 8
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_phong_eval.restype = C.c_double
        L.orc_phong_eval.argtypes = [C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_phong_sample.restype = C.c_double
        L.orc_phong_sample.argtypes = [C.c_double, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                       C.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _spectrum(dst, spec, keep):
    if spec is None:
        dst.kind = 0
        dst.n = 0
        return
    if "gauss" in spec:
        terms = spec["gauss"]
        dst.kind = 1
        dst.n = len(terms)
        for i, (mu, sd, w) in enumerate(terms):
            dst.x[i], dst.s[i], dst.y[i] = mu, sd, w
    elif "pwl" in spec:
        knots = spec["pwl"]
        dst.kind = 2
        dst.n = len(knots)
        for i, (nm, v) in enumerate(knots):
            dst.x[i], dst.y[i] = nm, v
    elif "table" in spec:
        vals = np.ascontiguousarray(spec["table"], dtype=np.float64)
        keep.append(vals)
        dst.kind = 3
        dst.n = len(vals)
        dst.tab = vals.ctypes.data
    else:
        raise OracleError(f"unknown spectrum {spec}")


def make_scene(d):
    sc = Scene()
    keep = []   # tabulated spectra: arrays the struct points at, alive with it
    sc._keep = keep
    g = d["grid"]
    sc.n_bins, sc.lo_nm, sc.hi_nm = g["n_bins"], g["lo_nm"], g["hi_nm"]
    sc.natural_base = 1 if d.get("absorptivity_base", "decadic") == "natural" else 0
    sc.n_dyes = len(d["dyes"])
    for i, dy in enumerate(d["dyes"]):
        _spectrum(sc.dyes[i].absorption, dy["absorption"], keep)
        _spectrum(sc.dyes[i].emission, dy["emission"], keep)
        sc.dyes[i].epsilon = dy["epsilon"]
        sc.dyes[i].qy = dy["qy"]
    sc.n_media = len(d["media"])
    for i, md in enumerate(d["media"]):
        sc.media[i].sigma_s = md["sigma_s"]
        sc.media[i].sigma_a_bg = md["sigma_a_bg"]
        sc.media[i].ior = md.get("ior", 1.0)
        sc.media[i].n_dyes = len(md["dyes"])
        for j, (di, c) in enumerate(md["dyes"]):
            sc.media[i].dye[j] = di
            sc.media[i].conc[j] = c
    geo = d["geometry"]
    kind = geo["kind"]
    if kind == "slab":
        sc.geom, sc.z0, sc.z1 = 0, geo["z0"], geo["z1"]
    elif kind == "halfspace":
        sc.geom, sc.z0, sc.z1 = 1, geo["z0"], math.inf
    elif kind == "sphere":
        sc.geom = 2
        sc.center[:] = geo["center"]
        sc.radius = geo["radius"]
    elif kind == "infinite":
        sc.geom = 3
    elif kind == "box":
        sc.geom = 4
        sc.box_lo[:] = geo["lo"]
        sc.box_hi[:] = geo["hi"]
        sc.open_face = geo["open_face"]
        for f, w in enumerate(geo["walls"]):
            _spectrum(sc.walls[f], w, keep)
        sc.wall_gloss[:] = geo.get("wall_gloss", [0.0] * 6)
        sc.n_spheres = len(geo["spheres"])
        for i, sp in enumerate(geo["spheres"]):
            sc.spheres[i].center[:] = sp["center"]
            sc.spheres[i].radius = sp["radius"]
            sc.spheres[i].medium = sp["medium"]
    else:
        raise OracleError(f"unknown geometry {kind}")
    if kind != "box":
        sc.body_medium = geo["medium"]
    li = d["light"]
    lk = li["kind"]
    if lk == "beam":
        sc.light = 0
        sc.lpos[:] = li["pos"]
        sc.ldir[:] = li["dir"]
    elif lk == "point":
        sc.light = 1
        sc.lpos[:] = li["pos"]
    elif lk == "quad":
        sc.light = 2
        sc.lpos[:] = li["corner"]
        sc.lu[:] = li["u"]
        sc.lv[:] = li["v"]
    else:
        raise OracleError(f"unknown light {lk}")
    sc.n_lines = len(li["lines"])
    for i, (nm, p) in enumerate(li["lines"]):
        sc.line_nm[i] = nm
        sc.line_power[i] = p
    se = d["sensor"]
    if se["kind"] == "escape":
        sc.sensor = 0
    else:
        sc.sensor = 1
        sc.eye[:] = se["eye"]
        sc.look[:] = se["look"]
        sc.up[:] = se["up"]
        sc.fov_y_deg = se["fov_y_deg"]
        sc.width = se["width"]
        sc.height = se["height"]
    return sc


def make_run(r):
    ru = Run()
    ru.seed = r["seed"]
    ru.instance = r["instance"]
    ru.max_scatter = r["max_scatter"]
    ru.path_begin = r["path_begin"]
    ru.path_count = r["path_count"]
    ru.total_paths = r["total_paths"]
    ru.max_emissions = r["max_emissions"]
    ru.fluorescence_only = 1 if r["fluorescence_only"] else 0
    ru.excitation_scatter = 1 if r["excitation_scatter"] else 0
    ru.parity_batches = r["parity_batches"]
    ru.splat_rr = r["splat_rr"]
    ru.perturb_eta = r.get("perturb_eta", 0.0)
    ru.perturb_pattern = r.get("perturb_pattern", 0)
    return ru


def film_shape(scene, batches=1):
    n = scene["grid"]["n_bins"]
    se = scene["sensor"]
    if se["kind"] == "pinhole":
        return (batches, 2, se["height"], se["width"], n)
    return (batches, 2, 2, n)


def n_params(scene):
    return lib().orc_n_params(C.byref(make_scene(scene)))


def _ptr(a):
    return None if a is None else a.ctypes.data


def render(scene, run, film=True, grad_film=None, records=False, record_grad=False,
           max_vertices=0, film_out=None):
    """Run the oracle walk.  Returns a dict with 'film' (fp64, film_shape),
    'tallies' (uint64[20]), optionally 'grad', 'records', 'record_grad'.
    film_out: a C-contiguous fp64 array of the film's shape to accumulate into
    (returned as 'film') instead of a new zeroed film."""
    L = lib()
    sc = make_scene(scene)
    ru = make_run(run)
    B = max(1, run["parity_batches"])
    out = {}
    if film_out is not None:
        if (film_out.dtype != np.float64 or not film_out.flags.c_contiguous
                or film_out.shape != film_shape(scene, B)):
            raise OracleError("film_out must be a C-contiguous float64 array of the film's shape")
        f = film_out
    else:
        f = np.zeros(film_shape(scene, B), np.float64) if film else None
    t = np.zeros(N_TALLIES, np.uint64)
    g = None
    gf = None
    np_ = L.orc_n_params(C.byref(sc))
    if grad_film is not None:
        gf = np.ascontiguousarray(grad_film, dtype=np.float64)
        if gf.size != int(np.prod(film_shape(scene, B))):
            raise OracleError("grad_film has the wrong size")
        g = np.zeros(np_, np.float64)
    rec = np.zeros(run["path_count"], RECORD_DTYPE) if records else None
    rg = np.zeros((run["path_count"], np_), np.float64) if record_grad else None
    rc = L.orc_render(C.byref(sc), C.byref(ru), _ptr(f), _ptr(t), _ptr(gf), _ptr(g),
                      _ptr(rec), _ptr(rg), max_vertices)
    if rc != 0:
        raise OracleError(L.orc_last_error().decode())
    out["film"] = f
    out["tallies"] = t
    if g is not None:
        out["grad"] = g
    if rec is not None:
        out["records"] = rec
    if rg is not None:
        out["record_grad"] = rg
    return out


INT_FIELDS = ("n_vertices", "n_scatter", "n_emit", "exit_code", "lambda", "comp")


def replay_condition(scene, run, max_vertices=0, grad_film=None, camera=False,
                     eta=2.0 ** -23, patterns=(1, 2), scale=1.0):
    """Per-path records and their condition numbers, for replay comparisons.

    Renders the path range plainly and again with every position and direction
    the walk computes scaled coordinate-wise by 1 +- eta (eta = one fp32 ulp at
    1; signs hashed per path, vertex and coordinate; one run per pattern).  For
    each record field the condition number is the largest change between a
    perturbed run and the plain one, divided by eta times the field's size
    (positions: at least `scale`; directions: at least 1; splat sums and
    per-path gradients: their own magnitude, gradients as vectors).  A walk
    whose every vertex state carries a relative error d moves that field by
    about kappa * d.  Paths whose integer outcome changes under the
    perturbation are flagged `unstable` (a decision within about eta of its
    threshold).  Returns a dict: 'records', optionally 'record_grad', and
    'kappa_pos', 'kappa_dir', 'kappa_splat', optionally 'kappa_grad' (each
    float64[path_count]), 'unstable' (bool[path_count])."""
    def once(extra):
        r = dict(run, **extra)
        if camera:
            return render_camera(scene, r, records=True, max_vertices=max_vertices)
        return render(scene, r, grad_film=grad_film, records=True,
                      record_grad=grad_film is not None, max_vertices=max_vertices)

    base = once({})
    rec = base["records"]
    n = len(rec)
    out = {"records": rec, "unstable": np.zeros(n, bool),
           "kappa_pos": np.zeros(n), "kappa_dir": np.zeros(n), "kappa_splat": np.zeros(n)}
    g0 = base.get("record_grad")
    if g0 is not None:
        out["record_grad"] = g0
        out["kappa_grad"] = np.zeros(n)
    for pat in patterns:
        o = once({"perturb_eta": eta, "perturb_pattern": pat})
        pr = o["records"]
        for f in INT_FIELDS:
            out["unstable"] |= pr[f].astype(np.int64) != rec[f].astype(np.int64)
        for f, floor in (("pos", scale), ("dir", 1.0)):
            k = (np.abs(pr[f] - rec[f]) / (eta * np.maximum(np.abs(rec[f]), floor))).max(1)
            out["kappa_" + f] = np.maximum(out["kappa_" + f], k)
        d = np.abs(pr["splat_sum"] - rec["splat_sum"])
        a = np.abs(rec["splat_sum"])
        k = np.where(d == 0, 0.0, d / (eta * np.maximum(a, 1e-300)))
        out["kappa_splat"] = np.maximum(out["kappa_splat"], k)
        if g0 is not None:
            d = np.linalg.norm(o["record_grad"] - g0, axis=1)
            a = np.linalg.norm(g0, axis=1)
            k = np.where(d == 0, 0.0, d / (eta * np.maximum(a, 1e-300)))
            out["kappa_grad"] = np.maximum(out["kappa_grad"], k)
    return out


def phong_eval(n, wi, wo, nrm):
    """The glossy wall lobe over rho, (n+2)/(2 pi) cos^n(alpha) (test hook)."""
    a = [np.ascontiguousarray(v, np.float64) for v in (wi, wo, nrm)]
    return lib().orc_phong_eval(float(n), *[x.ctypes.data for x in a])


def phong_sample(n, wi, nrm, ua, ub):
    """A direction drawn from the glossy lobe and its throughput factor (test hook)."""
    a = [np.ascontiguousarray(v, np.float64) for v in (wi, nrm)]
    wo = np.zeros(3)
    f = lib().orc_phong_sample(float(n), a[0].ctypes.data, a[1].ctypes.data, float(ua), float(ub),
                               wo.ctypes.data)
    return wo, f


def camera_paths(scene, spp):
    """Path count of a camera-side render with spp samples per (pixel, bin)."""
    se = scene["sensor"]
    return spp * se["height"] * se["width"] * scene["grid"]["n_bins"]


def render_camera(scene, run, film=True, records=False, max_vertices=0):
    """Run the camera-side estimator (paths from the eye, light connected at
    each collision in a dye medium).  run["total_paths"] must be
    camera_paths(scene, spp).  Returns 'film' (fp64, film_shape; component 1
    only), 'tallies' and optionally 'records'."""
    L = lib()
    sc = make_scene(scene)
    ru = make_run(run)
    B = max(1, run["parity_batches"])
    f = np.zeros(film_shape(scene, B), np.float64) if film else None
    t = np.zeros(N_TALLIES, np.uint64)
    rec = np.zeros(run["path_count"], RECORD_DTYPE) if records else None
    rc = L.orc_render_camera(C.byref(sc), C.byref(ru), _ptr(f), _ptr(t), _ptr(rec),
                             max_vertices)
    if rc != 0:
        raise OracleError(L.orc_last_error().decode())
    out = {"film": f, "tallies": t}
    if rec is not None:
        out["records"] = rec
    return out


def tallies_dict(t):
    return {n: int(v) for n, v in zip(TALLY_NAMES, t)}


def tables(scene):
    L = lib()
    sc = make_scene(scene)
    N = scene["grid"]["n_bins"]
    nd = max(1, len(scene["dyes"]))
    nm = max(1, len(scene["media"]))
    lam = np.zeros(N)
    ahat = np.zeros((nd, N))
    pmf = np.zeros((nd, N))
    cdf = np.zeros((nd, N))
    st = np.zeros((nm, N))
    sa = np.zeros((nm, MAX_MEDIUM_DYES, N))
    rho = np.zeros((6, N))
    lb = np.zeros(MAX_LINES, np.int32)
    rc = L.orc_tables(C.byref(sc), _ptr(lam), _ptr(ahat), _ptr(pmf), _ptr(cdf), _ptr(st),
                      _ptr(sa), _ptr(rho), _ptr(lb))
    if rc != 0:
        raise OracleError(L.orc_last_error().decode())
    return {"lambda": lam, "a_hat": ahat, "emis_pmf": pmf, "emis_cdf": cdf,
            "sigma_t": st, "sigma_a": sa, "rho": rho,
            "line_bin": lb[:len(scene["light"]["lines"])]}


def philox(ctr, key):
    """Philox4x32-10 of the given counter (4 words) and key (2 words)."""
    c = np.asarray(ctr, np.uint32).copy()
    k = np.asarray(key, np.uint32).copy()
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o
