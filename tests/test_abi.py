"""CPU checks of the C ABI boundary: the library loads, exports every symbol
declared in include/fpt.h, its struct layouts match the Python mirror, and
descriptor validation rejects bad input before touching any device."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

import workloads
from paper_1706_03024_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpt.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fpt_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    syms = declared_symbols()
    assert len(syms) >= 17
    for s in syms:
        assert hasattr(L, s), s
    assert L.fpt_abi_version() == _abi.ABI_VERSION == 5
    assert L.fpt_status_str(-3) == b"out of memory"


def test_struct_layouts_match_header():
    d = tempfile.mkdtemp(prefix="abi_")
    exe = os.path.join(d, "layout")
    subprocess.run(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "pins", "abi_layout.c"), "-o", exe], check=True)
    out = dict(l.split() for l in subprocess.run([exe], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    assert int(out["fpt_spectrum"]) == C.sizeof(_abi.Spectrum)
    assert int(out["fpt_dye"]) == C.sizeof(_abi.Dye)
    assert int(out["fpt_medium"]) == C.sizeof(_abi.Medium)
    assert int(out["fpt_sphere"]) == C.sizeof(_abi.Sphere)
    assert int(out["fpt_scene_desc"]) == C.sizeof(_abi.SceneDesc)
    assert int(out["fpt_run"]) == C.sizeof(_abi.Run)
    assert int(out["fpt_tune"]) == C.sizeof(_abi.Tune)
    assert int(out["fpt_path_record"]) == C.sizeof(_abi.PathRecord)
    assert int(out["off_geometry"]) == _abi.SceneDesc.geometry.offset
    assert int(out["off_light"]) == _abi.SceneDesc.light.offset
    assert int(out["off_sensor"]) == _abi.SceneDesc.sensor.offset
    assert int(out["off_fov"]) == _abi.SceneDesc.fov_y_deg.offset
    assert int(out["off_gloss"]) == _abi.SceneDesc.wall_gloss.offset
    assert int(out["off_splat_rr"]) == _abi.Run.splat_rr.offset


def _create_status(scene):
    d = _abi.scene_desc(scene)
    h = C.c_void_p()
    rc = _abi.lib().fpt_scene_create(C.byref(d), C.byref(h))
    if rc == 0:
        _abi.lib().fpt_scene_destroy(h)
    return rc, _abi.lib().fpt_last_error().decode()


@pytest.mark.parametrize("mutate,code", [
    (lambda s: s["dyes"][0].__setitem__("qy", 1.5), _abi.E_RANGE),
    (lambda s: s["dyes"][0].__setitem__("epsilon", -1.0), _abi.E_RANGE),
    (lambda s: s["media"][0].__setitem__("sigma_s", float("nan")), _abi.E_RANGE),
    (lambda s: s["media"][0].__setitem__("sigma_a_bg", -0.1), _abi.E_RANGE),
    (lambda s: s["media"][0].__setitem__("ior", 0.5), _abi.E_RANGE),
    (lambda s: s["dyes"][0].__setitem__("absorption", {"table": [1.0] * 100}), _abi.E_RANGE),
    (lambda s: s["dyes"][0].__setitem__("emission", {"table": [1.0] * 100 + [float("nan")]}),
     _abi.E_INVALID),
    (lambda s: s["media"][0].__setitem__("ior", 4.5), _abi.E_RANGE),
    (lambda s: s["light"].__setitem__("lines", [[900.0, 1.0]]), _abi.E_RANGE),
    (lambda s: s["light"].__setitem__("lines", [[490.0, 0.0]]), _abi.E_INVALID),
    (lambda s: s["grid"].__setitem__("n_bins", 1), _abi.E_RANGE),
    (lambda s: s["geometry"].__setitem__("z1", -1.0), _abi.E_INVALID),
    (lambda s: s["media"][0].__setitem__("dyes", [[3, 1.0]]), _abi.E_INVALID),
    (lambda s: s["dyes"][0].__setitem__("absorption", {"gauss": [[490.0, 0.0, 1.0]]}),
     _abi.E_INVALID),
    (lambda s: s.__setitem__("sensor", {"kind": "pinhole", "eye": [0, 0, 3], "look": [0, 0, 0],
                                        "up": [0, 1, 0], "fov_y_deg": 40, "width": 8,
                                        "height": 8}), _abi.E_UNSUPPORTED),
])
def test_invalid_slab_descriptors_rejected(mutate, code):
    s = workloads.slab_scene()
    mutate(s)
    rc, msg = _create_status(s)
    assert rc == code, msg
    assert msg


def test_invalid_box_descriptors_rejected():
    s = workloads.cornell_scene(8, 8)
    s["geometry"]["spheres"][1]["center"] = [-0.4, -0.79, -0.2]  # overlaps sphere 0
    assert _create_status(s)[0] == _abi.E_INVALID
    s = workloads.cornell_scene(8, 8)
    s["geometry"]["spheres"][0]["center"] = [-0.5, -0.8, -0.2]  # touches the floor
    assert _create_status(s)[0] == _abi.E_INVALID
    s = workloads.cornell_scene(8, 8)
    s["geometry"]["walls"][0] = workloads.pwl((300, 0.5), (800, 1.5))
    assert _create_status(s)[0] == _abi.E_RANGE
    s = workloads.cornell_scene(8, 8)
    s["sensor"]["eye"] = [0.0, 0.0, 0.0]
    assert _create_status(s)[0] == _abi.E_UNSUPPORTED
    s = workloads.cornell_scene(8, 8)
    s["media"][1]["ior"] = 1.5   # refracting sphere: no straight camera connection through it
    assert _create_status(s)[0] == _abi.E_UNSUPPORTED


def test_glossy_walls_rejected_where_unsupported():
    s = workloads.glossy_cornell_scene(8, 8)
    s["geometry"]["wall_gloss"][2] = -1.0
    assert _create_status(s)[0] == _abi.E_RANGE
    s = workloads.glossy_cornell_scene(8, 8)
    s["geometry"]["wall_gloss"][2] = 2e4
    assert _create_status(s)[0] == _abi.E_RANGE
    s = workloads.glossy_cornell_scene(8, 8)
    s["sensor"] = {"kind": "escape"}
    assert _create_status(s)[0] == _abi.E_UNSUPPORTED


def test_null_arguments_rejected():
    L = _abi.lib()
    h = C.c_void_p()
    assert L.fpt_scene_create(None, C.byref(h)) == _abi.E_INVALID
    r = _abi.run_struct(workloads.make_run(16))
    assert L.fpt_render(None, C.byref(r), None, None, None) == _abi.E_INVALID
    assert L.fpt_render_adjoint(None, C.byref(r), None, None, None, None) == _abi.E_INVALID
    assert L.fpt_render_camera(None, C.byref(r), None, None, None, 0, None) == _abi.E_INVALID
