"""GPU forward path vs the oracle and the closed forms (needs an MI355X).

Replay tests run both sides on identical Philox streams and compare per-path
records; statistical tests compare films from independent seeds bin by bin;
pins re-run the oracle's closed-form checks on the HIP path at larger sizes.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from replay import compare_records, oracle_replay
from stats import batch_z, binom_z, check_z, escape_z, multinomial_z

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


def _render(scene, run):
    import torch
    fpt = _fpt()
    sc = fpt.Scene(scene)
    t = fpt.new_tallies()
    film = sc.render(run, tallies=t)
    torch.cuda.synchronize()
    out = film.cpu().numpy().astype(np.float64), fpt.tallies_dict(t)
    sc.close()
    return out


def _records(scene, run, max_vertices=0):
    fpt = _fpt()
    sc = fpt.Scene(scene)
    rec, _ = sc.records(run, max_vertices=max_vertices)
    sc.close()
    return rec


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("name", ["slab", "cornell", "large"])
def test_tables_match_oracle(name):
    scene = {"slab": lambda: workloads.slab_scene(),
             "cornell": lambda: workloads.cornell_scene(8, 8),
             "large": lambda: workloads.large_scene(8, 8)}[name]()
    sc = _fpt().Scene(scene)
    g = sc.tables()
    o = oracle.tables(scene)
    sc.close()
    np.testing.assert_allclose(g["sigma_t"], o["sigma_t"].astype(np.float32), rtol=2.4e-7)
    np.testing.assert_allclose(g["emis_cdf"], o["emis_cdf"].astype(np.float32), rtol=2.4e-7,
                               atol=1e-30)
    assert np.all(g["emis_cdf"][:, -1] == 1.0)
    if scene["geometry"]["kind"] == "box":
        np.testing.assert_allclose(g["rho"], o["rho"].astype(np.float32), rtol=2.4e-7)
    np.testing.assert_array_equal(g["line_bin"], o["line_bin"])


# ------------------------------------------------------------------ plain slab
def test_slab_replay_all_paths():
    """Plain slab, all 2^16 paths, full length: every non-marginal path
    reproduces the oracle's vertex count, scatters, emissions, exit,
    wavelength and exit state (fp32 vs fp64, relative 1e-5 scaled by the
    path's condition number)."""
    scene, run = workloads.slab_config()
    g = _records(scene, run)
    rep = compare_records(g, oracle_replay(scene, run))
    print(rep)


@pytest.mark.parametrize("ior", [1.0, 1.33])
def test_slab_full_size_sampled(ior):
    """The benchmark's 2^22-path slab in its launch shape, index-matched and
    behind a water boundary: sampled path ranges replay against the oracle,
    and the escape film equals the exits."""
    import torch
    from paper_1706_03024_amd import autotune
    fpt = _fpt()
    scene, run = workloads.slab_config()
    scene["media"][0]["ior"] = ior
    n = 1 << 22
    run = dict(run, path_count=n, total_paths=n)
    sc = fpt.Scene(scene)
    autotune.autotune("slab-2^22", scene=sc, run=run, measure=False)  # the cached shape, if any
    t = fpt.new_tallies()
    film = sc.render(run, tallies=t)
    rec, _ = sc.records(run)
    torch.cuda.synchronize()
    td = fpt.tallies_dict(t)
    f = film.cpu().numpy().astype(np.float64)[0]
    sc.close()
    assert td["paths"] == n
    assert abs(f.sum() * n - (td["exit_esc_r"] + td["exit_esc_t"])) <= 1e-3 * n
    for begin in (0, n // 2 - 2048, n - 4096):
        sub = dict(run, path_begin=begin, path_count=4096)
        compare_records(rec[begin:begin + 4096], oracle_replay(scene, sub))


def test_slab_statistical_parity():
    """Independent seeds: GPU film (2^20 paths) vs oracle film (2^16 paths),
    per-bin multinomial z-scores."""
    scene, run = workloads.slab_config()
    ng, no = 1 << 20, 1 << 16
    g, tg = _render(scene, dict(run, seed=101, path_count=ng, total_paths=ng))
    o = oracle.render(scene, dict(run, seed=202, path_count=no, total_paths=no))
    check_z(escape_z(g[0], ng, o["film"][0], no), "slab film: GPU vs oracle")
    assert tg["paths"] == ng


def test_slab_same_seed_film_and_tallies():
    """Same seed: films and tallies agree up to the few marginal paths."""
    scene, run = workloads.slab_config()
    g, tg = _render(scene, run)
    o = oracle.render(scene, run)
    to = oracle.tallies_dict(o["tallies"])
    n = run["path_count"]
    for k in oracle.TALLY_NAMES:
        assert abs(tg[k] - to[k]) <= max(4, 1e-4 * max(to[k], 1)), (k, tg[k], to[k])
    assert np.abs(g - o["film"]).max() * n <= 8


def test_determinism_and_sharding():
    """Repeated renders are bit-identical; rendering [0,k) and [k,N) into the
    same film equals rendering [0,N) (integer escape tallies)."""
    import torch
    fpt = _fpt()
    scene, run = workloads.slab_config()
    sc = fpt.Scene(scene)
    t1, t2, t3 = fpt.new_tallies(), fpt.new_tallies(), fpt.new_tallies()
    f1 = sc.render(run, tallies=t1)
    f2 = sc.render(run, tallies=t2)
    k = 12345
    f3 = sc.render(dict(run, path_count=k), tallies=t3)
    sc.render(dict(run, path_begin=k, path_count=run["path_count"] - k), film=f3, tallies=t3)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(t1, t2)
    assert torch.equal(f1, f3) and torch.equal(t1, t3)
    sc.set_tune(block_threads=128, refill_lanes=48)
    t4 = fpt.new_tallies()
    f4 = sc.render(run, tallies=t4)
    torch.cuda.synchronize()
    assert torch.equal(f1, f4) and torch.equal(t1, t4)
    sc.close()


def test_conservation_identities():
    scene, run = workloads.slab_config()
    _, t = _render(scene, dict(run, path_count=1 << 18, total_paths=1 << 18))
    n = 1 << 18
    assert t["paths"] == n
    assert sum(t["exit_" + e] for e in oracle.EXIT_NAMES) == n
    assert t["dye_abs"] == t["emissions"] + t["exit_nonrad"] + t["exit_kcap"]
    s3 = workloads.t3_conservative_slab()
    f, t3 = _render(s3, workloads.make_run(n, seed=9))
    assert t3["exit_esc_r"] + t3["exit_esc_t"] + t3["exit_scap"] == n
    assert abs(f.sum() - (1 - t3["exit_scap"] / n)) < 1e-5


# ------------------------------------------------------------------ closed forms on the GPU
def test_gpu_beer_lambert_and_single_scatter():
    n = 1 << 20
    rec = _records(workloads.t1_beer_lambert(), workloads.make_run(n, seed=3))
    ballistic = np.sum((rec["exit_code"] == 1) & (rec["n_vertices"] == 2))
    assert abs(binom_z(ballistic, n, math.exp(-1.0))) < 4.5
    tau = 0.05
    rec = _records(workloads.t7_single_scatter(tau), workloads.make_run(n, seed=41))
    one = rec["n_scatter"] == 1
    R1, T1 = cf.single_scatter_slab(tau)
    assert abs(binom_z(np.sum(one & (rec["exit_code"] == 0)), n, R1)) < 4.5
    assert abs(binom_z(np.sum(one & (rec["exit_code"] == 1)), n, T1)) < 4.5


@pytest.mark.parametrize("albedo", [0.5, 0.99])
def test_gpu_infinite_medium_moments(albedo):
    n = 1 << 18
    rec = _records(workloads.t2_infinite(albedo, sigma_t=2.0), workloads.make_run(n, seed=11))
    ns = rec["n_scatter"].astype(float)
    assert abs(ns.mean() - albedo / (1 - albedo)) < 4.5 * math.sqrt(albedo) / (1 - albedo) / math.sqrt(n)
    r2 = (rec["pos"].astype(float) ** 2).sum(1)
    assert abs(r2.mean() - 2 / (2.0 * 2.0 * (1 - albedo))) < 4.5 * r2.std() / math.sqrt(n)


def test_gpu_quantum_yield_and_emission_shape():
    n = 1 << 18
    qy = 0.7
    _, t = _render(workloads.t4_infinite_dye(qy=qy),
                   workloads.make_run(n, seed=21, max_emissions=workloads.UNLIMITED_EMISSIONS))
    assert abs(binom_z(t["emissions"], t["dye_abs"], qy)) < 4.5
    rec = _records(workloads.t4_infinite_dye(qy=0.9), workloads.make_run(n, seed=22))
    em = rec[rec["n_emit"] == 1]
    hist = np.bincount(em["lambda"], minlength=101) / len(em)
    check_z(multinomial_z(hist, len(em), cf.emission_pmf(101, [(560, 30, 1)])),
            "GPU emission shape")


def test_gpu_dye_slab_closed_form():
    n = 1 << 20
    lx, d, conc, bg, qy = 490.0, 1.0, 20.0, 0.05, 0.8
    f, _ = _render(workloads.t6_dye_slab(lambda_x=lx, conc_uM=conc, sigma_a_bg=bg, d=d, qy=qy),
                   workloads.make_run(n, seed=31))
    lam = cf.grid_lambda(101)
    sa = cf.dye_sigma_a(lam, [(490, 20, 1)], 7e4, conc, 101)
    st = bg + sa
    R, T = cf.dye_slab_fluorescent_film(d, st[38], sa[38], qy, cf.emission_pmf(101, [(520, 25, 1)]), st)
    z = np.concatenate([multinomial_z(f[0, 1, 0], n, R), multinomial_z(f[0, 1, 1], n, T)])
    check_z(z, "GPU dye slab fluorescent film")


@pytest.mark.parametrize("albedo", [0.9, 0.99])
def test_gpu_halfspace_albedo(albedo):
    n = 1 << 19
    _, t = _render(workloads.t8_halfspace(albedo), workloads.make_run(n, seed=51))
    assert abs(binom_z(t["exit_esc_r"], n, cf.halfspace_albedo(albedo))) < 4.5


# ------------------------------------------------------------------ sphere body
def test_sphere_body_replay_and_parity():
    scene = workloads.sphere_scene()
    n = 1 << 14
    run = workloads.make_run(n, seed=5)
    compare_records(_records(scene, run), oracle_replay(scene, run, scale=0.5), scale=0.5)
    ng = 1 << 20
    g, _ = _render(scene, workloads.make_run(ng, seed=6))
    o = oracle.render(scene, workloads.make_run(n * 4, seed=7))
    check_z(escape_z(g[0], ng, o["film"][0], n * 4), "sphere body film")


# ------------------------------------------------------------------ camera scenes
def test_cornell_replay():
    """Box scene with pinhole splats: per-path replay of 2^15 paths, including
    the sum of each path's splat values."""
    scene = workloads.cornell_scene(32, 32)
    run = workloads.make_run(1 << 15, seed=4)
    rep = compare_records(_records(scene, run), oracle_replay(scene, run))
    print(rep)


def test_cornell_statistical_parity():
    """Batch-mean z-scores of the spectral film, independent seeds."""
    B = 32
    scene = workloads.cornell_scene(32, 32)
    g, _ = _render(scene, workloads.make_run(1 << 21, seed=10, parity_batches=B))
    o = oracle.render(scene, workloads.make_run(1 << 18, seed=11, parity_batches=B))["film"]
    z = batch_z(g, o)
    assert z.size > 500
    check_z(z, "Cornell film: GPU vs oracle", dof=B - 1)


def test_cornell_full_size_sampled():
    """Full 128x128, 2^20-path Cornell render in the benchmark's launch
    configuration: the film total equals the sum of every path's deposited
    values, and three sampled ranges of 4096 paths replay against the oracle
    over their first 256 vertices and at full length."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd import autotune
    scene, run = workloads.cornell_config()
    sc = fpt.Scene(scene)
    autotune.autotune("cornell-128-64spp", scene=sc, run=run, measure=False)  # the cached shape, if any
    film = sc.render(run)
    rec, _ = sc.records(run)
    torch.cuda.synchronize()
    total = float(film.double().sum())
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    N = run["path_count"]
    for begin in (0, N // 3, N - 4096):
        sub = dict(run, path_begin=begin, path_count=4096)
        g256, _ = sc.records(sub, max_vertices=256)
        print("256 vertices", compare_records(g256, oracle_replay(scene, sub, max_vertices=256)))
        print("full length", compare_records(rec[begin:begin + 4096], oracle_replay(scene, sub)))
    sc.close()


def test_large_scene_sampled_replay():
    """Large 5-sphere scene (301 bins, sigma_s up to 1000/mm), in the
    benchmark's launch shape: three sampled ranges of 4096 paths, first 256
    vertices, replay against the oracle."""
    from paper_1706_03024_amd import autotune
    scene, run = workloads.large_config()
    sc = _fpt().Scene(scene)
    autotune.autotune("large-512-1024spp", scene=sc, run=run, measure=False)  # the cached shape, if any
    for begin in (7, 123456789, run["path_count"] - 4096):
        sub = dict(run, path_begin=begin, path_count=4096)
        g, _ = sc.records(sub, max_vertices=256)
        print(compare_records(g, oracle_replay(scene, sub, max_vertices=256)))
    sc.close()


def test_large_scene_forward_film():
    """The benchmark's forward instantiation on the large scene (5 bimodal
    dye spheres, 301 bins, sigma_s up to 1000/mm, scatter cap 1e4) in its
    tuned launch shape, at 16x16 pixels: 128-vertex deep rounds, deferred
    connections and merged deposits.  The film, in 32 parity slices, agrees
    bin by bin with the oracle's film of independent paths (batch-mean z per
    film cell, per pixel summed over wavelength, and per 10-bin band summed
    over the image); on the same paths its total equals the sum of the
    replayed records' deposits and its integer tallies the oracle's."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd import autotune
    B = 32
    scene = workloads.large_scene(16, 16)
    _, big_run = workloads.large_config()
    sc = fpt.Scene(scene)
    autotune.autotune("large-512-1024spp", scene=sc, run=big_run, measure=False)
    run = workloads.make_run(1 << 25, seed=31, parity_batches=B)
    g = sc.render(run).cpu().numpy().astype(np.float64)
    same = workloads.make_run(1 << 22, seed=33)
    film = sc.render(same)
    rec, _ = sc.records(same)
    torch.cuda.synchronize()
    total = float(film.double().sum())
    sc.close()
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    # same paths on both sides: the integer tallies agree up to marginal paths,
    # among them the connections the kernel counts without evaluating (zero
    # transmittance inside the vertex's own sphere: hits, or roulette kills)
    fpt_sc = fpt.Scene(scene)
    for rr in (0.0, 0.05):
        small = workloads.make_run(1 << 16, seed=34, splat_rr=rr)
        tg = fpt.new_tallies()
        fpt_sc.render(small, tallies=tg)
        torch.cuda.synchronize()
        tg = fpt.tallies_dict(tg)
        to = oracle.tallies_dict(oracle.render(scene, small)["tallies"])
        for k in ("vertices", "splat_hit", "splat_miss", "splat_rr_kill", "emissions"):
            assert abs(tg[k] - to[k]) <= max(8, 1e-4 * to[k]), (rr, k, tg[k], to[k])
        assert to["splat_hit"] > 0 and (rr == 0.0 or to["splat_rr_kill"] > 0)
        # a third of the connections start deep inside the densest spheres
        assert tg["splat_opaque"] > 0.2 * (tg["splat_hit"] + tg["splat_rr_kill"])
    fpt_sc.close()
    o = oracle.render(scene, workloads.make_run(1 << 21, seed=32, parity_batches=B))["film"]
    z = batch_z(g, o)
    assert z.size > 1000
    check_z(z, "large scene film cells: GPU vs oracle", dof=B - 1)
    check_z(batch_z(g.sum(4), o.sum(4)), "large scene image (summed over wavelength)", dof=B - 1)
    band = lambda f: f[..., :300].reshape(f.shape[:-1] + (30, 10)).sum(-1).sum((2, 3))
    zb = batch_z(band(g), band(o))
    check_z(zb, "large scene spectrum in 10-bin bands (summed over the image)", dof=B - 1)


def test_splat_roulette_and_fluorescence_only():
    """Transmittance roulette keeps the film unbiased; fluorescence_only keeps
    only the emitted component.  Both match the oracle on the same streams."""
    scene = workloads.cornell_scene(32, 32)
    run = workloads.make_run(1 << 14, seed=12, splat_rr=0.05, fluorescence_only=True)
    compare_records(_records(scene, run), oracle_replay(scene, run))
    B = 32
    g, _ = _render(scene, workloads.make_run(1 << 21, seed=13, parity_batches=B, splat_rr=0.05))
    o = oracle.render(scene, workloads.make_run(1 << 18, seed=14, parity_batches=B))["film"]
    check_z(batch_z(g, o), "roulette film vs plain oracle film", dof=B - 1)


@pytest.mark.parametrize("scene_name", ["slab", "box"])
def test_block_rounds_are_width_independent(scene_name):
    """Long paths walk in wave blocks of 64, 32 or 16 lanes depending on how
    many share a wave, or 128 vertices per round when deep in a medium; the
    arithmetic is defined in 16-vertex chunks, so every launch shape, segment
    count and round width gives bit-identical integer tallies."""
    import torch
    fpt = _fpt()
    if scene_name == "slab":
        scene, run = workloads.slab_config()
        run = dict(run, path_count=1 << 18, total_paths=1 << 18)
    else:
        scene = workloads.cornell_scene(8, 8)
        scene["sensor"] = {"kind": "escape"}
        run = workloads.make_run(1 << 18, seed=3)
    sc = fpt.Scene(scene)
    outs = []
    for tune in ({"block_segments": 1}, {"block_segments": 4},
                 {"block_segments": 2, "block_threads": 64, "refill_lanes": 1},
                 {"block_segments": 4, "block_threads": 128, "refill_lanes": 40},
                 {"block_segments": 4, "wide_rounds": -1}, {"block_segments": 1, "wide_rounds": -1},
                 {"block_segments": 2, "wide_rounds": 2}):
        sc.set_tune(**tune)
        t = fpt.new_tallies()
        f = sc.render(run, tallies=t)
        torch.cuda.synchronize()
        outs.append((f.clone(), t.clone()))
    sc.close()
    for f, t in outs[1:]:
        assert torch.equal(t, outs[0][1])
        assert torch.equal(f, outs[0][0])




def test_spheres_in_line_forward_film():
    """Two dense spheres in line with the eye: connections from the far one
    cross the near one, so its occluder mask holds both spheres and the deep
    rounds' in-place evaluation takes the clear form over that mask, while
    the near sphere, occluded by itself only, takes the one-chord form.  In
    the Cornell box's tuned launch shape at 16x16 pixels the film agrees bin by
    bin with the oracle's (batch-mean z), and on the same paths its total equals
    the sum of the replayed records' deposits."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd import autotune
    scene = workloads.cornell_scene(16, 16)
    scene["geometry"]["spheres"] = [
        {"center": [0.0, -0.40, 0.35], "radius": 0.2, "medium": 2},   # near the eye
        {"center": [0.0, -0.50, -0.40], "radius": 0.2, "medium": 2},  # behind it, in line
    ]
    sc = fpt.Scene(scene)
    clear, occl = sc.connection_masks()
    assert clear == 3 and occl[0] == 1 and occl[1] == 3, (clear, occl)
    _, big_run = workloads.cornell_config()
    autotune.autotune("cornell-128-64spp", scene=sc, run=big_run, measure=False)
    B = 32
    g = sc.render(workloads.make_run(1 << 24, seed=41, parity_batches=B)).cpu().numpy().astype(np.float64)
    same = workloads.make_run(1 << 21, seed=43)
    t = fpt.new_tallies()
    film = sc.render(same, tallies=t)
    rec, _ = sc.records(same)
    torch.cuda.synchronize()
    total = float(film.double().sum())
    sc.close()
    assert abs(total - float(rec["splat_sum"].astype(np.float64).sum())) <= 1e-4 * total
    td = fpt.tallies_dict(t)
    # paths enter the spheres and walk long chains there (deep rounds); none is
    # deep enough for a zero-valued connection, so every full half of a deep
    # round connects in place
    assert td["crossings"] > 0 and td["splat_opaque"] == 0, td
    o = oracle.render(scene, workloads.make_run(1 << 22, seed=42, parity_batches=B))["film"]
    z = batch_z(g, o)
    assert z.size > 500, z.size  # chiefly the three excitation lines: emission is rare here
    check_z(z, "in-line spheres film: GPU vs oracle", dof=B - 1)

def test_large_scene_paths_are_schedule_independent():
    """At the large scene's full size (2^28 paths into the pinhole film) the
    launch shape and the timing of the path queue decide which paths share a
    wave, and with that which rounds walk each path (16, 32 or 64 lanes, or
    128-vertex deep rounds).  Every shape gives the same paths bit for bit, so
    every integer tally is identical, in repeated renders too.  Paths whose
    stop decision sits within an ulp of a tie (a flight ending at a sphere's
    surface; a few in 2^28) expose any difference between the rounding of the
    rounds' code paths: before their arithmetic was written out, one or two
    such paths per render walked differently from render to render.  The film
    is a sum of float atomics in no fixed order, so it agrees to rounding."""
    import torch
    fpt = _fpt()
    scene, run = workloads.large_config()
    sc = fpt.Scene(scene)
    base = {"block_min_vertices": 1}
    outs = []
    for tune in ({"block_threads": 256, "refill_lanes": 16, "block_segments": 4, "wide_rounds": 1},
                 {"block_threads": 256, "refill_lanes": 16, "block_segments": 4, "wide_rounds": 1},
                 {"block_segments": 1},
                 {"block_segments": 2, "block_threads": 128, "refill_lanes": 40},
                 {"block_segments": 4, "wide_rounds": -1},
                 {"block_segments": 4, "wide_rounds": 2, "block_threads": 64, "refill_lanes": 1}):
        sc.set_tune(**base, **tune)
        t = fpt.new_tallies()
        f = sc.render(run, tallies=t)
        torch.cuda.synchronize()
        outs.append((f.clone(), t.clone()))
        print("tune", tune, "vertices", int(t[1]), flush=True)
    sc.close()
    f0, t0 = outs[0]
    tol = 1e-5 * float(f0.abs().max())
    for f, t in outs[1:]:
        assert torch.equal(t, t0), (fpt.tallies_dict(t), fpt.tallies_dict(t0))
        assert torch.allclose(f, f0, rtol=1e-3, atol=tol)


def test_tabulated_spectra():
    """Tabulated spectra (one value per grid point, as measured spectra come):
    the Cornell scene with every spectrum sampled on its grid has the same fp32
    tables as the analytic one (within an ulp; identical in practice), and with
    identical tables every path is bit-identical to the analytic scene's, whose
    walk the oracle replay covers; the library keeps its own copy of the
    arrays."""
    fpt = _fpt()
    s = workloads.cornell_scene(16, 16)
    t = workloads.tabulated_scene(s)
    sa, st = fpt.Scene(s), fpt.Scene(t)
    ga, gt = sa.tables(), st.tables()
    for k in ("sigma_t", "emis_cdf", "rho"):
        np.testing.assert_allclose(gt[k], ga[k], rtol=2.4e-7, atol=1e-30)
    # the caller's arrays may change or go away after creation
    for arr in st._d._keep:
        arr[:] = 0.0
    np.testing.assert_array_equal(st.tables()["sigma_t"], gt["sigma_t"])
    run = workloads.make_run(1 << 15, seed=17)
    ra, _ = sa.records(run)
    rt, _ = st.records(run)
    sa.close()
    st.close()
    if all(np.array_equal(gt[k], ga[k]) for k in ("sigma_t", "emis_cdf", "rho")):
        assert np.array_equal(rt.view(np.uint32), ra.view(np.uint32))
    else:
        st = fpt.Scene(t)
        rt, _ = st.records(run, max_vertices=256)
        st.close()
        compare_records(rt, oracle_replay(t, run, max_vertices=256))
