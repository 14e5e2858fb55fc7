"""Pins of the CPU oracle against closed forms, invariants and a library routine.

Every test here runs on the CPU only.  Citations are to the paper
(arXiv 1706.03024): section / equation.
"""
from __future__ import annotations

import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from stats import binom_z, check_z, multinomial_z

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ RNG
@pytest.fixture(scope="module")
def rocrand_ref():
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "ref")
    src = os.path.join(HERE, "pins", "rocrand_philox_ref.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    src, "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    """Philox4x32-10 (counter-based RNG of every random decision) equals rocRAND's
    independent implementation on random counters and keys."""
    rng = np.random.default_rng(7)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] %= 2**30  # keeps rocRAND's offset = 4*(c0|c1<<32) below 2^64
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    ctr[:8] = 0
    ctr[8:16, 0] = np.arange(8)
    key[:4] = 0
    inp = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([list(map(int, l.split())) for l in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    mine = np.array([oracle.philox(c.astype(np.uint32), k.astype(np.uint32))
                     for c, k in zip(ctr, key)], dtype=np.uint64)
    assert ref.shape == (n, 4)
    np.testing.assert_array_equal(mine, ref)


# ------------------------------------------------------------------ tables
def test_tables_normalisation_and_units():
    """Sec. 4.1 / eq. 10 readings: absorption peak-normalised to 1 on the grid,
    emission an area-normalised PMF with CDF ending at exactly 1,
    sigma_a = ln10 * eps * c * 1e-7 * a_hat (1/mm), sigma_t = sigma_s + sigma_a (eq. 6)."""
    s = workloads.slab_scene()
    t = oracle.tables(s)
    N = 101
    lam = cf.grid_lambda(N)
    np.testing.assert_allclose(t["lambda"], lam, rtol=0, atol=1e-12)
    assert t["a_hat"][0].max() == 1.0
    assert t["emis_cdf"][0][-1] == 1.0
    assert np.all(np.diff(t["emis_cdf"][0]) >= 0)
    np.testing.assert_allclose(t["emis_pmf"][0].sum(), 1.0, rtol=0, atol=N * 2.3e-16)
    np.testing.assert_allclose(t["emis_pmf"][0], cf.emission_pmf(N, [(520, 25, 1)]),
                               rtol=1e-12)
    sa = cf.dye_sigma_a(lam, [(490, 20, 1)], 7e4, 10.0, N)
    np.testing.assert_allclose(t["sigma_a"][0, 0], sa, rtol=1e-12)
    # 490 nm is grid point 38; ln10 * 7e4 * 10 uM * 1e-7 = 0.16118 /mm at the peak
    assert t["line_bin"][0] == 38
    assert abs(t["sigma_a"][0, 0, 38] - 0.161181) < 1e-6
    np.testing.assert_allclose(t["sigma_t"][0], 10.0 + 0.01 + sa, rtol=1e-12)
    # natural-base reading is ln10 times smaller
    s2 = workloads.slab_scene()
    s2["absorptivity_base"] = "natural"
    t2 = oracle.tables(s2)
    np.testing.assert_allclose(t2["sigma_a"][0, 0] * math.log(10), t["sigma_a"][0, 0], rtol=1e-12)


def test_tables_walls_and_line_snapping():
    s = workloads.cornell_scene(8, 8)
    t = oracle.tables(s)
    lam = t["lambda"]
    # piecewise-linear walls reproduce their knots and interpolate linearly
    assert t["rho"][0][lam.tolist().index(580.0)] == pytest.approx(0.05)
    assert t["rho"][0][lam.tolist().index(620.0)] == pytest.approx(0.70)
    assert t["rho"][0][lam.tolist().index(600.0)] == pytest.approx(0.375)
    assert t["rho"][5].max() == 0.0  # open face
    assert list(t["line_bin"]) == [30, 50, 70]
    # ties go to the lower grid point
    s3 = workloads.slab_scene(lambda_x=302.5)
    assert oracle.tables(s3)["line_bin"][0] == 0
    s4 = workloads.slab_scene(lambda_x=302.6)
    assert oracle.tables(s4)["line_bin"][0] == 1


def test_invalid_descriptors_rejected():
    s = workloads.slab_scene()
    s["dyes"][0]["qy"] = 1.5
    with pytest.raises(oracle.OracleError):
        oracle.render(s, workloads.make_run(16))
    s = workloads.slab_scene(lambda_x=900.0)
    with pytest.raises(oracle.OracleError):
        oracle.render(s, workloads.make_run(16))
    s = workloads.slab_scene()
    s["media"][0]["sigma_s"] = -1.0
    with pytest.raises(oracle.OracleError):
        oracle.render(s, workloads.make_run(16))
    with pytest.raises(oracle.OracleError):
        oracle.render(workloads.slab_scene(), workloads.make_run(16, path_begin=8, total_paths=16))


# ------------------------------------------------------------------ P1 Beer-Lambert
def test_beer_lambert_ballistic_fraction():
    """Eq. 6: the fraction of beam photons crossing a slab of optical thickness
    tau without a collision is exp(-tau)."""
    n = 1 << 17
    s = workloads.t1_beer_lambert(d=1.0, sigma_s=0.5, sigma_a=0.5)
    o = oracle.render(s, workloads.make_run(n, seed=3), records=True)
    rec = o["records"]
    ballistic = np.sum((rec["exit_code"] == 1) & (rec["n_vertices"] == 2))
    assert abs(binom_z(ballistic, n, math.exp(-1.0))) < 4.5
    # absorption-only slab: the elastic T film bin equals exp(-tau) in expectation
    s2 = workloads.t1_beer_lambert(d=0.5, sigma_s=0.0, sigma_a=2.0)
    o2 = oracle.render(s2, workloads.make_run(n, seed=4))
    T = o2["film"][0, 0, 1, 38]
    assert abs(binom_z(T * n, n, math.exp(-1.0))) < 4.5


# ------------------------------------------------------------------ P2 infinite medium
@pytest.mark.parametrize("albedo", [0.5, 0.9, 0.99])
def test_infinite_medium_moments(albedo):
    """Infinite isotropic medium: collisions per path are geometric with mean
    1/(1-a); scatters have mean a/(1-a); at absorption <r^2> = 2/(sigma_t sigma_a)."""
    n = 1 << 15
    s = workloads.t2_infinite(albedo, sigma_t=2.0)
    o = oracle.render(s, workloads.make_run(n, seed=11), records=True)
    rec = o["records"]
    ns = rec["n_scatter"].astype(float)
    mean_s = albedo / (1 - albedo)
    sd_s = math.sqrt(albedo) / (1 - albedo)
    assert abs(ns.mean() - mean_s) < 4.5 * sd_s / math.sqrt(n)
    assert np.all(rec["exit_code"] == 2)  # background absorption ends every path
    assert np.all(rec["n_vertices"] == rec["n_scatter"] + 2)
    r2 = (rec["pos"] ** 2).sum(1)
    sig_t, sig_a = 2.0, 2.0 * (1 - albedo)
    assert abs(r2.mean() - 2 / (sig_t * sig_a)) < 4.5 * r2.std() / math.sqrt(n)
    # isotropic directions: E[w] = 0, E[w_z^2] = 1/3
    wz = rec["dir"][:, 2]
    assert abs(wz.mean()) < 4.5 * math.sqrt(1 / 3 / n)
    assert abs((wz ** 2).mean() - 1 / 3) < 4.5 * math.sqrt(4 / 45 / n)


# ------------------------------------------------------------------ P3 conservation
def test_conservation_and_vertex_identity():
    """Every path ends in exactly one exit; the vertex tally equals the sum of
    per-path vertex counts; a non-absorbing slab loses nothing."""
    n = 1 << 13
    s = workloads.t3_conservative_slab(tau=10.0)
    o = oracle.render(s, workloads.make_run(n, seed=5), records=True)
    t = oracle.tallies_dict(o["tallies"])
    assert t["paths"] == n
    assert sum(t["exit_" + e] for e in oracle.EXIT_NAMES) == n
    assert t["exit_esc_r"] + t["exit_esc_t"] + t["exit_scap"] == n
    assert t["vertices"] == int(o["records"]["n_vertices"].sum())
    f = o["film"][0]
    assert f.sum() == pytest.approx(1.0 - t["exit_scap"] / n, abs=1e-12)
    s2, r2 = workloads.slab_config()
    r2 = dict(r2, path_count=4096, total_paths=4096)
    o2 = oracle.render(s2, r2)
    t2 = oracle.tallies_dict(o2["tallies"])
    assert sum(t2["exit_" + e] for e in oracle.EXIT_NAMES) == 4096
    assert t2["dye_abs"] == t2["emissions"] + t2["exit_nonrad"] + t2["exit_kcap"]


def test_sharding_is_exact():
    """[0,k) + [k,N) == [0,N): the counter-based RNG makes path ranges independent."""
    s, r = workloads.slab_config()
    N = 4096
    full = oracle.render(s, dict(r, path_count=N, total_paths=N))
    a = oracle.render(s, dict(r, path_count=1000, total_paths=N))
    b = oracle.render(s, dict(r, path_begin=1000, path_count=N - 1000, total_paths=N))
    np.testing.assert_array_equal(full["tallies"], a["tallies"] + b["tallies"])
    np.testing.assert_allclose(full["film"], a["film"] + b["film"], rtol=0, atol=1e-15)


# ------------------------------------------------------------------ P4 / P5 quantum yield, emission shape
def test_quantum_yield_ratio():
    """Sec. 4.1: a dye absorption emits with probability QY; in an infinite
    non-scattering medium with unlimited emissions the number of emissions per
    path is geometric with mean QY/(1-QY)."""
    n = 1 << 15
    qy = 0.7
    s = workloads.t4_infinite_dye(qy=qy)
    o = oracle.render(s, workloads.make_run(n, seed=21, max_emissions=workloads.UNLIMITED_EMISSIONS),
                      records=True)
    t = oracle.tallies_dict(o["tallies"])
    assert abs(binom_z(t["emissions"], t["dye_abs"], qy)) < 4.5
    ne = o["records"]["n_emit"].astype(float)
    assert abs(ne.mean() - qy / (1 - qy)) < 4.5 * math.sqrt(qy) / (1 - qy) / math.sqrt(n)
    assert t["exit_nonrad"] == n


def test_emission_spectrum_shape():
    """Eq. 10 and sec. 2.1: the re-emitted wavelength follows the normalised
    emission spectrum, whatever the excitation wavelength."""
    n = 1 << 16
    for lx in (400.0, 490.0, 600.0):
        s = workloads.t4_infinite_dye(qy=0.9)
        s["light"]["lines"] = [[lx, 1.0]]
        o = oracle.render(s, workloads.make_run(n, seed=int(lx)), records=True)
        rec = o["records"]
        em = rec[rec["n_emit"] == 1]
        assert np.all(rec[rec["n_emit"] == 1]["exit_code"] == 4)  # K=1: next absorption kills
        hist = np.bincount(em["lambda"], minlength=101) / len(em)
        p = cf.emission_pmf(101, [(560, 30, 1)])
        check_z(multinomial_z(hist, len(em), p), f"emission shape at {lx} nm")


# ------------------------------------------------------------------ P6 non-scattering dye slab
@pytest.mark.parametrize("lx", [450.0, 490.0, 530.0])
def test_dye_slab_fluorescent_film(lx):
    """Non-scattering dye slab: the first-collision law (eq. 6), the dye share
    sigma_a,d/sigma_t, QY and the emission PMF (eq. 10) with uncollided escape
    give the fluorescent reflected and transmitted spectra in closed form; the
    elastic transmission is exp(-sigma_t d) at the beam wavelength."""
    n = 1 << 17
    d, conc, bg, qy = 1.0, 20.0, 0.05, 0.8
    s = workloads.t6_dye_slab(lambda_x=lx, conc_uM=conc, sigma_a_bg=bg, d=d, qy=qy)
    o = oracle.render(s, workloads.make_run(n, seed=31))
    N = 101
    lam = cf.grid_lambda(N)
    k = int(round((lx - 300) / 5))
    sa = cf.dye_sigma_a(lam, [(490, 20, 1)], 7e4, conc, N)
    st = bg + sa
    pmf = cf.emission_pmf(N, [(520, 25, 1)])
    R, T = cf.dye_slab_fluorescent_film(d, st[k], sa[k], qy, pmf, st)
    f = o["film"][0]
    z = np.concatenate([multinomial_z(f[1, 0], n, R), multinomial_z(f[1, 1], n, T)])
    check_z(z, f"dye slab fluorescent film at {lx} nm")
    T_el = math.exp(-st[k] * d)
    assert abs(binom_z(f[0, 1, k] * n, n, T_el)) < 4.5
    t = oracle.tallies_dict(o["tallies"])
    p_em = qy * sa[k] / st[k] * (1 - math.exp(-st[k] * d))
    assert abs(binom_z(t["emissions"], n, p_em)) < 4.5


# ------------------------------------------------------------------ P7 single scattering
def test_single_scatter_slab():
    """Thin isotropic slab: paths with exactly one scatter leaving each face
    match the single-scattering integrals."""
    n = 1 << 18
    tau = 0.05
    s = workloads.t7_single_scatter(tau=tau)
    o = oracle.render(s, workloads.make_run(n, seed=41), records=True)
    rec = o["records"]
    one = rec["n_scatter"] == 1
    r1 = np.sum(one & (rec["exit_code"] == 0))
    t1 = np.sum(one & (rec["exit_code"] == 1))
    R1, T1 = cf.single_scatter_slab(tau)
    assert abs(binom_z(r1, n, R1)) < 4.5
    assert abs(binom_z(t1, n, T1)) < 4.5


# ------------------------------------------------------------------ P8 half-space albedo
def test_h_function_solver():
    """The H-function solver against its zeroth-moment identity
    int_0^1 H = (2/w)(1 - sqrt(1-w)) and the tabulated conservative H(1) = 2.9078."""
    for w in (0.5, 0.9, 0.99, 1.0):
        _, (x, wt, H) = cf.chandrasekhar_h(w, [1.0])
        assert abs((wt * H).sum() - 2 / w * (1 - math.sqrt(1 - w))) < 2e-4
    h1, _ = cf.chandrasekhar_h(1.0, [1.0])
    assert abs(h1[0] - 2.9078) < 2e-3


@pytest.mark.parametrize("albedo", [0.9, 0.99])
def test_halfspace_albedo(albedo):
    """Semi-infinite isotropic medium under a normal beam: total reflectance
    1 - H(1) sqrt(1 - a) (long multiple-scattering walks)."""
    n = 1 << 15
    s = workloads.t8_halfspace(albedo)
    o = oracle.render(s, workloads.make_run(n, seed=51))
    t = oracle.tallies_dict(o["tallies"])
    assert t["exit_scap"] == 0
    R = cf.halfspace_albedo(albedo)
    assert abs(binom_z(t["exit_esc_r"], n, R)) < 4.5


def test_tabulated_spectra_reproduce_the_analytic_scene():
    """Tabulated spectra are read on the grid points: the Cornell scene with
    every dye spectrum and wall reflectance sampled on its grid has the same
    tables (to the rounding of evaluating the same Gaussians in another
    language) and walks every path the same way."""
    s = workloads.cornell_scene(8, 8)
    t = workloads.tabulated_scene(s)
    ta, tb = oracle.tables(s), oracle.tables(t)
    for k in ta:
        np.testing.assert_allclose(np.asarray(tb[k], float), np.asarray(ta[k], float),
                                   rtol=1e-13, atol=1e-300)
    run = workloads.make_run(1 << 12, seed=6)
    a = oracle.render(s, run, records=True)
    b = oracle.render(t, run, records=True)
    assert np.array_equal(a["records"]["exit_code"], b["records"]["exit_code"])
    assert np.array_equal(a["records"]["n_vertices"], b["records"]["n_vertices"])
    np.testing.assert_allclose(b["film"], a["film"], rtol=1e-9, atol=1e-300)


def test_32bit_path_ids():
    """Path ids are the 32-bit first counter word: a job may hold 2^32 paths
    (its last ids render, each escape weighing 1/2^32), but one call may not
    walk all 2^32 of them."""
    s, r = workloads.slab_config()
    tail = dict(r, path_begin=(1 << 32) - 100, path_count=100, total_paths=1 << 32)
    o = oracle.render(s, tail)
    t = oracle.tallies_dict(o["tallies"])
    assert t["paths"] == 100
    assert abs(o["film"].sum() * 2.0 ** 32 - (t["exit_esc_r"] + t["exit_esc_t"])) < 1e-6
    with pytest.raises(oracle.OracleError):
        oracle.render(s, dict(r, path_begin=0, path_count=1 << 32, total_paths=1 << 32))
    with pytest.raises(oracle.OracleError):
        oracle.render(s, dict(r, path_count=16, total_paths=(1 << 32) + 1))
