"""GPU camera-side estimator vs the oracle (needs an MI355X).

Replay: both sides draw identical Philox streams per path, so non-marginal
paths agree in every integer outcome and, to fp32 rounding, in exit state and
deposit.  Films: element by element against the oracle on the same paths, and
batch-mean z-scores against the GPU forward walk with direct excitation (the
two estimators' common target).  Edge cases: sub-ranges, empty runs, shape
errors, the benchmark's full-size launch on sampled ranges."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from replay import TINY, compare_records, oracle_replay
from stats import check_z
from test_oracle_camera_side import direct_scene, shadow_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _fpt():
    import paper_1706_03024_amd as fpt
    return fpt


def camera_run(scene, spp, seed, B=1, **kw):
    return workloads.make_run(oracle.camera_paths(scene, spp), seed=seed, parity_batches=B, **kw)


def _camera(scene, run, records=False, max_vertices=0):
    import torch
    fpt = _fpt()
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    film = sc.render_camera(run, tallies=t)
    rec = sc.camera_records(run, max_vertices=max_vertices) if records else None
    torch.cuda.synchronize()
    out = film.cpu().numpy().astype(np.float64), fpt.tallies_dict(t), rec
    sc.close()
    return out


def _film_close(g, o, grec, cond, scene, run, rtol=1e-5, margin=2e-6):
    """Element-wise film agreement on the same paths.  A camera path deposits
    its whole sum into one cell (its sample's slice, pixel and bin), so each
    cell is a sum of known per-path deposits; the cell may differ from the
    oracle's by what its paths may differ (rtol * max(1, kappa) of each
    deposit, all of a marginal path's) plus the rounding of its fp32 atomic
    sums."""
    assert np.all(g[:, 0] == 0.0)
    N = scene["grid"]["n_bins"]
    W, H = scene["sensor"]["width"], scene["sensor"]["height"]
    B = max(1, run.get("parity_batches", 1))
    pid = run["path_begin"] + np.arange(run["path_count"], dtype=np.int64)
    k, pix, smp = pid % N, (pid // N) % (W * H), pid // (N * W * H)
    cell = (((smp % B) * 2 + 1) * (W * H) + pix) * N + k
    orc = cond["records"]
    a = np.abs(grec["splat_sum"].astype(np.float64))
    b = np.abs(orc["splat_sum"])
    marg = (orc["margin"] < margin) | cond["unstable"]
    per = np.where(marg, a + b, rtol * np.maximum(1.0, cond["kappa_splat"]) * np.maximum(a, b))
    allow = np.bincount(cell, per + 2.0 ** -22 * a, minlength=g.size).reshape(g.shape)
    d = np.abs(g - o)
    bad = np.nonzero(d > allow + TINY)
    assert bad[0].size == 0, (bad[0].size, d[bad][:5], allow[bad][:5])
    return float(np.max(d / np.maximum(allow, TINY)))


@pytest.mark.parametrize("make_scene", [direct_scene, shadow_scene])
def test_camera_replay_and_film(make_scene):
    """Every path of an 8x8, 26-bin render with 4 samples: records replay
    against the oracle; the film matches element by element and equals the
    sum of the records' deposits."""
    scene = make_scene()
    run = camera_run(scene, 4, seed=21)
    g, gt, grec = _camera(scene, run, records=True)
    o = oracle.render_camera(scene, run)
    cond = oracle_replay(scene, run, camera=True)
    print(compare_records(grec, cond))
    print("film deviation / allowance", _film_close(g, o["film"], grec, cond, scene, run))
    assert abs(g.sum() - float(grec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * g.sum()
    ot = oracle.tallies_dict(o["tallies"])
    assert gt["paths"] == ot["paths"] == run["path_count"]
    for k in ("vertices", "scatters", "wall_reflect", "crossings", "splat_hit"):
        assert abs(gt[k] - ot[k]) <= 1e-3 * max(ot[k], 1000), (k, gt[k], ot[k])


# Camera paths in the dense Cornell spheres walk up to a few thousand steps;
# replays of these scenes compare the first 512 vertices of each path.
DENSE_VERTICES = 512


def test_camera_replay_cornell_dense():
    """The benchmark's dense Cornell spheres (sigma_s 50-200/mm, 101 bins):
    4096 sampled paths per range replay against the oracle (first 512
    vertices)."""
    scene = workloads.cornell_scene(16, 16)
    run = camera_run(scene, 2, seed=22)
    fpt = _fpt()
    sc = fpt.Scene(scene)
    rec = sc.camera_records(run, max_vertices=DENSE_VERTICES)
    sc.close()
    n = run["path_count"]
    for begin in (0, n // 2 - 2048, n - 4096):
        sub = dict(run, path_begin=begin, path_count=4096)
        cond = oracle_replay(scene, sub, max_vertices=DENSE_VERTICES, camera=True)
        print(compare_records(rec[begin:begin + 4096], cond))


def test_camera_matches_gpu_forward_direct_excitation():
    """The GPU's two estimators of the same film component: forward walk with
    direct excitation and K = 1, and the camera-side walk (16x16, 51 bins)."""
    import torch
    fpt = _fpt()
    scene = direct_scene(width=16, n_bins=51)
    B = 32
    sc = fpt.Scene(scene)
    fwd = sc.render(workloads.make_run(1 << 26, seed=31, excitation_scatter=False,
                                       max_emissions=1, parity_batches=B))
    cam = sc.render_camera(camera_run(scene, 256, seed=32, B=B))
    torch.cuda.synchronize()
    ff = fwd.cpu().numpy().astype(np.float64)[:, 1]
    fc = cam.cpu().numpy().astype(np.float64)[:, 1]
    sc.close()

    def z(a, b):
        va, vb = a.var(0, ddof=1) / B, b.var(0, ddof=1) / B
        return (a.mean(0) - b.mean(0)) / np.sqrt(va + vb), b.mean(0)

    zt, _ = z(ff.sum(axis=(1, 2, 3)), fc.sum(axis=(1, 2, 3)))
    assert abs(zt) < 4.0
    zs, m = z(ff.sum(axis=(1, 2)), fc.sum(axis=(1, 2)))
    check_z(zs[m > 1e-2 * m.max()], "spectrum", dof=B - 1)
    zi, m = z(ff.sum(axis=3), fc.sum(axis=3))
    check_z(zi[m > 1e-2 * m.max()], "image", dof=B - 1)


def test_forward_direct_excitation_replay():
    """The forward walk without excitation scattering (paths end at their
    first scatter or wall reflection before emitting) replays the oracle."""
    scene = direct_scene(width=16, n_bins=51)
    run = workloads.make_run(1 << 15, seed=33, excitation_scatter=False, max_emissions=1)
    fpt = _fpt()
    sc = fpt.Scene(scene)
    rec, _ = sc.records(run)
    sc.close()
    print(compare_records(rec, oracle_replay(scene, run)))
    assert np.sum(rec["exit_code"] == 8) > 0


def test_camera_ranges_and_edges():
    """Disjoint sub-ranges add up to the whole render (records identical,
    film to fp32 rounding); an empty range is a no-op; a total that is not a
    whole number of samples, a missing output and an escape scene are
    rejected."""
    import torch
    fpt = _fpt()
    scene = direct_scene(width=8, n_bins=26)
    run = camera_run(scene, 3, seed=41)
    n = run["path_count"]
    sc = fpt.Scene(scene)
    whole = sc.render_camera(run)
    part = sc.new_film()
    cut = n // 3 + 7
    sc.render_camera(dict(run, path_count=cut), film=part)
    sc.render_camera(dict(run, path_begin=cut, path_count=n - cut), film=part)
    sc.render_camera(dict(run, path_begin=n, path_count=0), film=part)
    ra = sc.camera_records(run)
    rb = np.concatenate([sc.camera_records(dict(run, path_count=cut)),
                         sc.camera_records(dict(run, path_begin=cut, path_count=n - cut))])
    torch.cuda.synchronize()
    assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))
    a, b = whole.cpu().numpy(), part.cpu().numpy()
    np.testing.assert_allclose(b, a, rtol=1e-5, atol=1e-6 * a.max())
    with pytest.raises(Exception):
        sc.render_camera(dict(run, total_paths=n + 1, path_count=16))
    from paper_1706_03024_amd import _abi
    import ctypes as C
    r = _abi.run_struct(run)
    assert _abi.lib().fpt_render_camera(sc.handle, C.byref(r), None, None, None, 0, None) == \
        _abi.E_INVALID
    sc.close()
    slab = fpt.Scene(workloads.slab_scene())
    r = _abi.run_struct(workloads.make_run(64))
    buf = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    assert _abi.lib().fpt_render_camera(slab.handle, C.byref(r), C.c_void_p(buf.data_ptr()),
                                        None, None, 0, None) == _abi.E_UNSUPPORTED
    slab.close()


def test_camera_full_size_sampled():
    """The benchmark's camera workload (Cornell 128x128, 101 bins, 4 samples
    per pixel and bin) in its launch configuration: sampled ranges replay
    against the oracle (first 512 vertices) and the film total equals the sum
    of the records' deposits."""
    import torch
    fpt = _fpt()
    scene, run = workloads.camera_config()
    sc = fpt.Scene(scene)
    film = sc.render_camera(run)
    rec = sc.camera_records(run)
    torch.cuda.synchronize()
    total = float(film.double().sum())
    assert total > 0.0
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    n = run["path_count"]
    for begin in (0, n // 3, n - 2048):
        sub = dict(run, path_begin=begin, path_count=2048)
        g = sc.camera_records(sub, max_vertices=DENSE_VERTICES)
        cond = oracle_replay(scene, sub, max_vertices=DENSE_VERTICES, camera=True)
        print(compare_records(g, cond))
    sc.close()


def test_camera_launch_shape_independent():
    """Whether and when a path walks in wave rounds depends only on the path
    (24 vertices inside a sphere), never on the launch: records are identical
    bit for bit across block sizes, refill thresholds and occupancy, films
    agree to the order of their fp32 atomics."""
    import torch
    fpt = _fpt()
    scene = workloads.cornell_scene(16, 16)
    run = camera_run(scene, 2, seed=51)
    out = []
    for tune in ({}, {"block_threads": 64, "refill_lanes": 8, "blocks_per_cu": 1},
                 {"block_threads": 128, "refill_lanes": 60}):
        sc = fpt.Scene(scene)
        if tune:
            sc.set_tune(**tune)
        film = sc.render_camera(run)
        rec = sc.camera_records(run)
        torch.cuda.synchronize()
        out.append((film.cpu().numpy(), rec))
        sc.close()
    assert np.sum(out[0][1]["n_vertices"] > 200) > 0   # some paths did walk in rounds
    for film, rec in out[1:]:
        assert np.array_equal(rec.view(np.uint32), out[0][1].view(np.uint32))
        np.testing.assert_allclose(film, out[0][0], rtol=1e-5, atol=1e-7 * out[0][0].max())
