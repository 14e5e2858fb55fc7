"""Launch-shape autotuning with a JSON cache.

fpt_autotune times candidate shapes (block size, refill threshold, wave-block
trigger, and for batches the work-item size) on the device and returns the
fastest; results never depend on the shape.  The library owns the JSON cache
(keyed by the workload's name and the device's architecture and compute-unit
count); this module only passes its path and applies the result.
"""
from __future__ import annotations

import ctypes as C
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


def autotune(name, scene=None, run=None, batch=None, cache_path=DEFAULT_CACHE, force=False,
             measure=True):
    """fpt_autotune for workload `name`: the cached shape for this device, or
    a measured one (written to the cache) unless measure=False, in which case
    an uncached workload returns None (library defaults).  Applies the shape
    to `scene` (plain render) or returns it for a new Batch."""
    out = _abi.Tune()
    ms = C.c_float()
    flags = (_abi.TUNE_FORCE if force else 0) | (0 if measure else _abi.TUNE_CACHED_ONLY)
    path = cache_path.encode() if cache_path else None
    if batch is not None:
        check(lib().fpt_autotune(None, None, batch.handle, path, name.encode(), flags,
                                 C.byref(out), C.byref(ms)))
    elif scene is not None:
        r = _abi.run_struct(run)
        check(lib().fpt_autotune(scene.handle, C.byref(r), None, path, name.encode(), flags,
                                 C.byref(out), C.byref(ms)))
    else:   # a lookup only
        check(lib().fpt_autotune(None, None, None, path, name.encode(),
                                 flags | _abi.TUNE_CACHED_ONLY, C.byref(out), C.byref(ms)))
        measure = False
    best = {f: int(getattr(out, f)) for f in FIELDS}
    best["ms"] = float(ms.value)
    if not measure and best["ms"] == 0.0 and not any(best[f] for f in FIELDS):
        return None
    if scene is not None:
        scene.set_tune(**{f: best.get(f, 0) for f in FIELDS})
    return best
