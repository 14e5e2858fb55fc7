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
