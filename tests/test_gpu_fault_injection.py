"""Allocation failures during scene and batch creation (FPT_FAULT_INJECT=N
makes the N-th allocation of one creation call fail as out of memory): each
call returns FPT_E_NOMEM with nothing left allocated on the device, and once N
passes the number of allocations the call succeeds.  No GPU fault is involved:
the library sees a failed allocation and takes its own error path."""
from __future__ import annotations

import os

import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    os.environ.pop("FPT_FAULT_INJECT", None)


def _free():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _sweep(make, close):
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import _abi
    obj = make()            # warm up: the runtime's own first-use allocations
    close(obj)
    base = _free()
    failures = 0
    for n in range(1, 64):
        os.environ["FPT_FAULT_INJECT"] = str(n)
        try:
            obj = make()
        except fpt.FptError as e:
            assert e.status == _abi.E_NOMEM, (n, str(e))
            failures += 1
            # the same failure again and again: nothing may accumulate
            for _ in range(7):
                with pytest.raises(fpt.FptError):
                    make()
            assert base - _free() < (2 << 20), (n, base - _free())
            continue
        os.environ.pop("FPT_FAULT_INJECT")
        close(obj)
        assert base - _free() < (2 << 20)
        return failures
    raise AssertionError("creation never succeeded")


@pytest.mark.parametrize("name", ["cornell", "slab"])
def test_scene_creation_fails_cleanly(name):
    import paper_1706_03024_amd as fpt
    scene = workloads.cornell_scene(16, 16) if name == "cornell" else workloads.slab_scene()
    n = _sweep(lambda: fpt.Scene(scene), lambda s: s.close())
    # the scene object, tables, queue, partials (+ counters or deferred slices), staging
    assert n >= 5


def test_batch_creation_fails_cleanly():
    import paper_1706_03024_amd as fpt
    scenes = [workloads.slab_scene(conc_uM=c) for c in (1.0, 10.0)]
    runs = [workloads.make_run(1 << 12, seed=1, instance=i) for i in range(2)]
    n = _sweep(lambda: fpt.Batch(scenes, runs), lambda b: b.close())
    assert n >= 7
