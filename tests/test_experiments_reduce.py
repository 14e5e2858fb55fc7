"""The SPD reductions of the experiment sweeps (host tensors; no GPU)."""
from __future__ import annotations

import numpy as np
import torch

from paper_1706_03024_amd import experiments as ex


def test_fluorescent_spd_and_normalisation():
    rng = np.random.default_rng(5)
    films = torch.tensor(rng.random((4, 2, 2, 7)), dtype=torch.float32)
    films[2] = 0.0
    spd = ex.fluorescent_spd(films)
    np.testing.assert_array_equal(spd.numpy(), (films[:, 1, 0] + films[:, 1, 1]).numpy())
    nz = ex.normalized(spd)
    for i in range(4):
        if i == 2:
            assert (nz[i] == 0).all()
        else:
            assert abs(float(nz[i].max()) - 1.0) < 1e-7
            np.testing.assert_allclose(nz[i].numpy(), (spd[i] / spd[i].max()).numpy(), rtol=1e-6)


def test_pinhole_spd_averages_lit_pixels():
    film = torch.zeros((2, 2, 3, 4, 5))
    film[0, 1, 0, 0] = torch.tensor([1.0, 2.0, 3.0, 0.0, 0.0])
    film[1, 1, 0, 0] = torch.tensor([1.0, 0.0, 0.0, 0.0, 0.0])
    film[1, 1, 2, 3] = torch.tensor([0.0, 0.0, 1.0, 1.0, 0.0])
    film[0, 0, 1, 1] = 100.0  # component 0 is ignored
    np.testing.assert_allclose(ex.pinhole_spd(film).numpy(), [1.0, 1.0, 2.0, 0.5, 0.0])
    assert (ex.pinhole_spd(torch.zeros((1, 2, 2, 2, 3))) == 0).all()


def test_rebin_keeps_totals_and_maps_points():
    f = torch.arange(501, dtype=torch.float64)[None] * 0.5 + 1.0
    r = ex.rebin(f, 5)
    assert r.shape == (1, 101)
    assert abs(float(r.sum()) - float(f.sum())) < 1e-9
    # an interior coarse point collects the five fine points centred on it
    assert float(r[0, 10]) == float(f[0, 48:53].sum())
    # a point shared by two coarse cells goes half to each
    g = torch.zeros((1, 9), dtype=torch.float64)
    g[0, 2] = 1.0
    np.testing.assert_array_equal(ex.rebin(g, 4).numpy(), [[0.5, 0.5, 0.0]])


def test_fine_grid_oracle_rebins_to_coarse():
    """The slab on a 1-nm grid (501 points), rebinned, against the 101-point
    grid: the film per bin scales with the bin width and the fluorescent
    and elastic spectra agree bin by bin (independent seeds)."""
    import oracle
    import workloads
    from stats import check_z, escape_z
    n = 1 << 15
    fine = oracle.render(workloads.slab_scene(n_bins=501), workloads.make_run(n, seed=51))["film"][0]
    coarse = oracle.render(workloads.slab_scene(n_bins=101), workloads.make_run(n, seed=52))["film"][0]
    fr = ex.rebin(torch.tensor(fine), 5).numpy()
    check_z(escape_z(fr, n, coarse, n), "1-nm grid rebinned vs 5-nm grid (oracle)")
