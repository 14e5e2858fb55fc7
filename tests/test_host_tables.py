"""Scene creation through the C ABI for every workload the tests and the
benchmark use: validation and the fp64 table build run on the host first, so
on a machine without a GPU every valid scene gets as far as the device query
(FPT_E_DEVICE) and every invalid one is refused before it.  Run plainly by the
CPU suite and, by test_sanitizers.py, against an address- and
undefined-behaviour-sanitised build of the host library."""
from __future__ import annotations

import ctypes as C

import pytest

import workloads
from paper_1706_03024_amd import _abi


def _scenes():
    out = {
        "slab": workloads.slab_scene(),
        "cornell": workloads.cornell_scene(16, 16),
        "glossy": workloads.glossy_cornell_scene(16, 16),
        "large": workloads.large_scene(16, 16),
        "maximal": workloads.maximal_scene(),
        "maximal_1024": workloads.maximal_scene(n_bins=1024),
        "tabulated": workloads.tabulated_scene(workloads.cornell_scene(8, 8)),
        "sphere": workloads.sphere_scene(),
        "halfspace": workloads.t8_halfspace(0.9),
        "infinite": workloads.t4_infinite_dye(),
        "dielectric": workloads.t11_dielectric_sphere_point(1.5),
        "validation": workloads.validation_scene(),
    }
    scenes, _ = workloads.batch_config()
    out["batch_0"] = scenes[0]
    out["batch_1023"] = scenes[-1]
    return out


@pytest.mark.parametrize("name", sorted(_scenes()))
def test_valid_scenes_build_their_tables(name):
    d = _abi.scene_desc(_scenes()[name])
    h = C.c_void_p()
    rc = _abi.lib().fpt_scene_create(C.byref(d), C.byref(h))
    msg = _abi.lib().fpt_last_error().decode()
    if rc == _abi.OK:
        _abi.lib().fpt_scene_destroy(h)
    else:
        assert rc == _abi.E_DEVICE and "device" in msg, (rc, msg)  # no GPU here


def test_scene_destroy_accepts_null():
    _abi.lib().fpt_scene_destroy(None)
    _abi.lib().fpt_batch_destroy(None)
