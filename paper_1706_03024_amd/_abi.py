"""ctypes mirror of include/fpt.h and the loader of libfpt.so.

Argument marshalling only: every step of the transport runs in the HIP
library.  Importing this module does not need a GPU; calling into the
library does.  A missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# a sanitizer build of the same sources may stand in for it (tests only)
LIB_PATH = os.environ.get("FPT_LIBRARY") or os.path.join(_HERE, "libfpt.so")

MAX_TERMS = 16
MAX_DYES = 8
MAX_MEDIA = 8
MAX_MEDIUM_DYES = 4
MAX_SPHERES = 8
MAX_LINES = 8
MAX_BINS = 1024
MAX_GRAD_PARAMS = 16
N_TALLIES = 21

OK, E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SPECTRUM_GAUSS_MIX, SPECTRUM_PIECEWISE_LINEAR, SPECTRUM_TABULATED = 1, 2, 3
GEOM = {"slab": 0, "halfspace": 1, "sphere": 2, "infinite": 3, "box": 4}
LIGHT = {"beam": 0, "point": 1, "quad": 2}
SENSOR = {"escape": 0, "pinhole": 1}
FLAG_FLUORESCENCE_ONLY = 1
FLAG_NO_EXCITATION_SCATTER = 2

EXIT_NAMES = ["esc_r", "esc_t", "bg", "nonrad", "kcap", "scap", "wall", "light", "excscat",
              "trunc"]
TALLY_NAMES = ["paths", "vertices", "scatters", "dye_abs", "emissions", "wall_reflect",
               "crossings", "splat_hit", "splat_miss", "splat_rr_kill"] + \
              ["exit_" + n for n in EXIT_NAMES] + ["splat_opaque"]


class FptError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fpt error {status}: {msg}")
        self.status = status


class Spectrum(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32),
                ("center_nm", C.c_double * MAX_TERMS), ("value", C.c_double * MAX_TERMS),
                ("width_nm", C.c_double * MAX_TERMS), ("table", C.c_void_p)]


class Dye(C.Structure):
    _fields_ = [("absorption", Spectrum), ("emission", Spectrum),
                ("epsilon_M_cm", C.c_double), ("qy", C.c_double)]


class Medium(C.Structure):
    _fields_ = [("sigma_s_mm", C.c_double), ("sigma_a_bg_mm", C.c_double),
                ("n_dyes", C.c_int32), ("dye", C.c_int32 * MAX_MEDIUM_DYES),
                ("conc_uM", C.c_double * MAX_MEDIUM_DYES), ("ior", C.c_double)]


class Sphere(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("radius", C.c_double), ("medium", C.c_int32),
                ("pad", C.c_int32)]


class SceneDesc(C.Structure):
    _fields_ = [
        ("n_bins", C.c_int32), ("absorptivity_base", C.c_int32),
        ("lo_nm", C.c_double), ("hi_nm", C.c_double),
        ("n_dyes", C.c_int32), ("n_media", C.c_int32),
        ("dyes", Dye * MAX_DYES), ("media", Medium * MAX_MEDIA),
        ("geometry", C.c_int32), ("body_medium", C.c_int32),
        ("slab_z0", C.c_double), ("slab_z1", C.c_double),
        ("body_center", C.c_double * 3), ("body_radius", C.c_double),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("open_face", C.c_int32), ("n_spheres", C.c_int32),
        ("walls", Spectrum * 6), ("spheres", Sphere * MAX_SPHERES),
        ("light", C.c_int32), ("n_lines", C.c_int32),
        ("light_pos", C.c_double * 3), ("light_dir", C.c_double * 3),
        ("light_u", C.c_double * 3), ("light_v", C.c_double * 3),
        ("line_nm", C.c_double * MAX_LINES), ("line_power", C.c_double * MAX_LINES),
        ("sensor", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
        ("eye", C.c_double * 3), ("look", C.c_double * 3), ("up", C.c_double * 3),
        ("fov_y_deg", C.c_double), ("wall_gloss", C.c_double * 6),
    ]


class Run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("path_begin", C.c_uint64), ("path_count", C.c_uint64),
                ("total_paths", C.c_uint64), ("instance", C.c_uint32),
                ("max_scatter", C.c_uint32), ("max_emissions", C.c_uint32),
                ("flags", C.c_uint32), ("parity_batches", C.c_uint32), ("pad", C.c_uint32),
                ("splat_rr", C.c_double)]


class Tune(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_lanes", C.c_int32), ("chunk_paths", C.c_int32),
                ("block_min_vertices", C.c_int32), ("block_segments", C.c_int32),
                ("wide_rounds", C.c_int32)]


class PathRecord(C.Structure):
    _fields_ = [("n_vertices", C.c_uint32), ("n_scatter", C.c_uint32), ("n_emit", C.c_uint32),
                ("exit_code", C.c_uint32), ("lambda_", C.c_int32), ("comp", C.c_int32),
                ("region", C.c_int32), ("pad", C.c_int32), ("pos", C.c_float * 3),
                ("dir", C.c_float * 3), ("splat_sum", C.c_float), ("pad2", C.c_float)]


RECORD_WORDS = C.sizeof(PathRecord) // 4
ABI_VERSION = 5
TUNE_FORCE, TUNE_CACHED_ONLY = 1, 2

_lib = None


def lib():
    """Load libfpt.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FptError(E_DEVICE, f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "fpt_abi_version": (C.c_uint32, []),
        "fpt_status_str": (C.c_char_p, [C.c_int32]),
        "fpt_last_error": (C.c_char_p, []),
        "fpt_scene_create": (C.c_int32, [C.POINTER(SceneDesc), C.POINTER(vp)]),
        "fpt_scene_destroy": (None, [vp]),
        "fpt_scene_set_params": (C.c_int32, [vp, vp, vp, vp, vp]),
        "fpt_film_shape": (C.c_int32, [vp, C.c_uint32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
        "fpt_grad_param_count": (C.c_int32, [vp]),
        "fpt_scene_set_tune": (C.c_int32, [vp, C.POINTER(Tune)]),
        "fpt_scene_set_timing": (C.c_int32, [vp, C.c_int32]),
        "fpt_scene_timing": (C.c_int32, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "fpt_scene_timing_each": (C.c_int32, [vp, C.c_int32, C.POINTER(C.c_int32), vp, vp]),
        "fpt_render": (C.c_int32, [vp, C.POINTER(Run), vp, vp, vp]),
        "fpt_render_noalloc": (C.c_int32, [vp, C.POINTER(Run), vp, vp, vp]),
        "fpt_render_adjoint": (C.c_int32, [vp, C.POINTER(Run), vp, vp, vp, vp]),
        "fpt_render_records": (C.c_int32, [vp, C.POINTER(Run), vp, C.c_uint32, vp, vp, vp]),
        "fpt_render_camera": (C.c_int32, [vp, C.POINTER(Run), vp, vp, vp, C.c_uint32, vp]),
        "fpt_scene_tables": (C.c_int32, [vp, vp, vp, vp, vp]),
        "fpt_scene_connection_masks": (C.c_int32, [vp, vp, vp]),
        "fpt_batch_create": (C.c_int32, [C.POINTER(SceneDesc), C.POINTER(Run), C.c_int32,
                                         C.POINTER(Tune), C.POINTER(vp)]),
        "fpt_batch_render": (C.c_int32, [vp, vp, vp, vp]),
        "fpt_batch_destroy": (None, [vp]),
        "fpt_autotune": (C.c_int32, [vp, C.POINTER(Run), vp, C.c_char_p, C.c_char_p, C.c_uint32,
                                     C.POINTER(Tune), C.POINTER(C.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.fpt_abi_version() != ABI_VERSION:
        raise FptError(E_INVALID, "libfpt ABI version mismatch")
    _lib = L
    return L


def check(status):
    if status != OK:
        raise FptError(status, lib().fpt_last_error().decode())


# ---------------------------------------------------------------- marshalling
def _spectrum(dst, spec, keep):
    if spec is None:
        dst.kind = 0
        dst.n = 0
        return
    if "gauss" in spec:
        dst.kind = SPECTRUM_GAUSS_MIX
        dst.n = len(spec["gauss"])
        for i, (mu, sd, w) in enumerate(spec["gauss"]):
            dst.center_nm[i], dst.width_nm[i], dst.value[i] = mu, sd, w
    elif "pwl" in spec:
        dst.kind = SPECTRUM_PIECEWISE_LINEAR
        dst.n = len(spec["pwl"])
        for i, (nm, v) in enumerate(spec["pwl"]):
            dst.center_nm[i], dst.value[i] = nm, v
    elif "table" in spec:
        vals = np.ascontiguousarray(spec["table"], dtype=np.float64)
        keep.append(vals)
        dst.kind = SPECTRUM_TABULATED
        dst.n = len(vals)
        dst.table = vals.ctypes.data
    else:
        raise FptError(E_INVALID, f"unknown spectrum {spec!r}")


def scene_desc(d):
    """Scene dictionary (see the workloads module) -> fpt_scene_desc.  The
    struct keeps the arrays of tabulated spectra alive (attribute _keep); the
    library copies them at fpt_scene_create / fpt_batch_create."""
    s = SceneDesc()
    keep = []
    s._keep = keep
    g = d["grid"]
    s.n_bins, s.lo_nm, s.hi_nm = g["n_bins"], g["lo_nm"], g["hi_nm"]
    s.absorptivity_base = 1 if d.get("absorptivity_base", "decadic") == "natural" else 0
    s.n_dyes = len(d["dyes"])
    for i, y in enumerate(d["dyes"]):
        _spectrum(s.dyes[i].absorption, y["absorption"], keep)
        _spectrum(s.dyes[i].emission, y["emission"], keep)
        s.dyes[i].epsilon_M_cm = y["epsilon"]
        s.dyes[i].qy = y["qy"]
    s.n_media = len(d["media"])
    for i, m in enumerate(d["media"]):
        s.media[i].sigma_s_mm = m["sigma_s"]
        s.media[i].sigma_a_bg_mm = m["sigma_a_bg"]
        s.media[i].ior = m.get("ior", 1.0)
        s.media[i].n_dyes = len(m["dyes"])
        for j, (di, c) in enumerate(m["dyes"]):
            s.media[i].dye[j] = di
            s.media[i].conc_uM[j] = c
    geo = d["geometry"]
    s.geometry = GEOM[geo["kind"]]
    if geo["kind"] == "slab":
        s.slab_z0, s.slab_z1 = geo["z0"], geo["z1"]
    elif geo["kind"] == "halfspace":
        s.slab_z0 = geo["z0"]
    elif geo["kind"] == "sphere":
        s.body_center[:] = geo["center"]
        s.body_radius = geo["radius"]
    elif geo["kind"] == "box":
        s.box_lo[:] = geo["lo"]
        s.box_hi[:] = geo["hi"]
        s.open_face = geo["open_face"]
        for f, w in enumerate(geo["walls"]):
            _spectrum(s.walls[f], w, keep)
        s.wall_gloss[:] = geo.get("wall_gloss", [0.0] * 6)
        s.n_spheres = len(geo["spheres"])
        for i, sp in enumerate(geo["spheres"]):
            s.spheres[i].center[:] = sp["center"]
            s.spheres[i].radius = sp["radius"]
            s.spheres[i].medium = sp["medium"]
    if geo["kind"] != "box":
        s.body_medium = geo["medium"]
    li = d["light"]
    s.light = LIGHT[li["kind"]]
    if li["kind"] == "quad":
        s.light_pos[:] = li["corner"]
        s.light_u[:] = li["u"]
        s.light_v[:] = li["v"]
    else:
        s.light_pos[:] = li["pos"]
        if li["kind"] == "beam":
            s.light_dir[:] = li["dir"]
    s.n_lines = len(li["lines"])
    for i, (nm, p) in enumerate(li["lines"]):
        s.line_nm[i] = nm
        s.line_power[i] = p
    se = d["sensor"]
    s.sensor = SENSOR[se["kind"]]
    if se["kind"] == "pinhole":
        s.eye[:] = se["eye"]
        s.look[:] = se["look"]
        s.up[:] = se["up"]
        s.fov_y_deg = se["fov_y_deg"]
        s.width = se["width"]
        s.height = se["height"]
    return s


def run_struct(r):
    """Run dictionary -> fpt_run."""
    ru = Run()
    ru.seed = r["seed"]
    ru.path_begin = r["path_begin"]
    ru.path_count = r["path_count"]
    ru.total_paths = r["total_paths"]
    ru.instance = r["instance"]
    ru.max_scatter = r["max_scatter"]
    ru.max_emissions = r["max_emissions"]
    ru.flags = (FLAG_FLUORESCENCE_ONLY if r.get("fluorescence_only") else 0) | \
        (0 if r.get("excitation_scatter", True) else FLAG_NO_EXCITATION_SCATTER)
    ru.parity_batches = r.get("parity_batches", 1)
    ru.splat_rr = r.get("splat_rr", 0.0)
    return ru
