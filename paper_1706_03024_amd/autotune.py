"""Launch-shape autotuning with a JSON cache.

fpt_autotune times candidate shapes (block size, refill threshold, wave-block
trigger, and for batches the work-item size) on the device and returns the
fastest; results never depend on the shape.  The cache is keyed by the
workload's name and the device's architecture and compute-unit count.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import torch

from . import _abi
from ._abi import check, lib

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
FIELDS = ("block_threads", "blocks_per_cu", "refill_lanes", "chunk_paths", "block_min_vertices",
          "block_segments", "wide_rounds")


def device_tag():
    """Architecture and compute-unit count of the current device (the
    marketing name is not always reported, e.g. under a profiler)."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.gcnArchName.split(':')[0]}x{p.multi_processor_count}cu"


def _key(name):
    return f"{name}@{device_tag()}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(name, scene=None, run=None, batch=None, cache_path=DEFAULT_CACHE, force=False,
             measure=True):
    """Returns the tune dict for `name`, measuring it if the cache lacks it
    (unless measure=False: then the library defaults, returned as None), and
    applies it to `scene` (plain render) or returns it for a new Batch."""
    cache = _load(cache_path)
    key = _key(name)
    if key in cache and not force:
        best = cache[key]
    elif not measure:
        return None
    else:
        out = _abi.Tune()
        ms = C.c_float()
        if batch is not None:
            check(lib().fpt_autotune(None, None, batch.handle, C.byref(out), C.byref(ms)))
        else:
            r = _abi.run_struct(run)
            check(lib().fpt_autotune(scene.handle, C.byref(r), None, C.byref(out), C.byref(ms)))
        best = {f: int(getattr(out, f)) for f in FIELDS}
        best["ms"] = float(ms.value)
        cache[key] = best
        try:
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    if scene is not None:
        scene.set_tune(**{f: best.get(f, 0) for f in FIELDS})
    return best
