"""fpt_render_noalloc (the allocation-free forward render) against fpt_render
through the C ABI: two calls in a row, the second on a smaller input, for a
pinhole box scene (deferred connections in the static scratch) and an escape
slab (escape counters in the static scratch).  Tallies are integers and must
be identical; escape films are integer counts scaled once, so identical too;
camera films are the same deposits summed by fp32 atomics in another order,
so each cell agrees to fp32 summation rounding.  The calls allocate no device
memory."""
from __future__ import annotations

import ctypes as C

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


def _pair(sc, run):
    """(film, tallies) of fpt_render and of fpt_render_noalloc, each called
    directly through the C ABI on the current stream."""
    import torch
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import _abi
    B = max(1, run.get("parity_batches", 1))
    r = _abi.run_struct(run)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for name in ("fpt_render", "fpt_render_noalloc"):
        film = sc.new_film(B)
        t = fpt.new_tallies()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        _abi.check(getattr(_abi.lib(), name)(sc.handle, C.byref(r), C.c_void_p(film.data_ptr()),
                                               C.c_void_p(t.data_ptr()), s))
        torch.cuda.synchronize()
        if name == "fpt_render_noalloc":
            assert torch.cuda.mem_get_info()[0] == free0
        out.append((film.cpu().numpy().astype(np.float64), t.cpu().numpy()))
    return out


def test_noalloc_matches_render_camera_scene():
    import paper_1706_03024_amd as fpt
    scene = workloads.cornell_scene(32, 32)
    sc = fpt.Scene(scene)
    for n, seed, B in ((1 << 20, 3, 4), (1 << 14, 4, 1)):   # second call: smaller input
        (fa, ta), (fb, tb) = _pair(sc, workloads.make_run(n, seed=seed, parity_batches=B))
        assert np.array_equal(ta, tb)
        assert fpt.tallies_dict(ta)["paths"] == n and fpt.tallies_dict(ta)["splat_hit"] > 0
        # sums of the same positive deposits in another order: fp32 rounding of
        # a sum of k terms grows like sqrt(k) ulps, well inside 1e-5 relative
        tol = 1e-5 * np.maximum(fa, fb) + 1e-30
        assert np.all(np.abs(fa - fb) <= tol), float(np.max(np.abs(fa - fb) / tol))
        assert np.count_nonzero(fa) == np.count_nonzero(fb) > 0
    sc.close()


def test_noalloc_matches_render_escape_slab():
    import paper_1706_03024_amd as fpt
    scene, run = workloads.slab_config()
    sc = fpt.Scene(scene)
    for n, seed, B in ((1 << 20, 7, 64), (1 << 12, 8, 1)):
        (fa, ta), (fb, tb) = _pair(sc, dict(run, path_count=n, total_paths=n, seed=seed,
                                             parity_batches=B))
        assert np.array_equal(ta, tb) and np.array_equal(fa, fb)
        assert fpt.tallies_dict(ta)["paths"] == n
    sc.close()
