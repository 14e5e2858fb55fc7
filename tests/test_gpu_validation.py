"""The paper's spectral validation (sec. 6, Figs. 6-7) on GPU renders.

The paper renders fluorescent samples under single-line excitation and checks
that the spectrum the image records, averaged over the pixels that receive
fluorescence and peak-normalised, follows the dye's emission spectrum, whatever
the excitation wavelength.  Here: one sphere of a single synthetic Gaussian dye
(weak: 5 uM, little scattering) in a box with black walls, fluorescence-only
pinhole film, reduced by experiments.pinhole_spd and normalized.

* Against the oracle: the same reduction of the oracle's own film, bin by bin
  by batch means over 32 parity slices.
* Against the emission spectrum: the only thing between the emitted and the
  recorded spectrum is reabsorption by the dye on the way out, at most
  1 - exp(-sigma_a,max 2r) of the light at any wavelength; the normalised SPD
  lies within that of the normalised emission PMF (plus 4 standard errors).
* Excitation invariance (Fig. 7): at two excitation lines the normalised SPDs
  agree within the same bound.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from stats import batch_z, check_z

pytestmark = pytest.mark.gpu

B = 32
CONC = 5.0
SIGMA_S = 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _gpu_spd(lambda_x, n, seed):
    """(normalised SPD, per-slice spectra [B][N], standard error of the
    normalised SPD) of a GPU render, through experiments.pinhole_spd."""
    import torch
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import experiments as ex
    scene = workloads.validation_scene(lambda_x=lambda_x, conc_uM=CONC, sigma_s=SIGMA_S)
    sc = fpt.Scene(scene)
    film = sc.render(workloads.make_run(n, seed=seed, parity_batches=B, fluorescence_only=True))
    spd = ex.normalized(ex.pinhole_spd(film))
    torch.cuda.synchronize()
    sc.close()
    f = film.double()[:, 1].sum((1, 2)).cpu().numpy()          # [B][N]
    tot = f.sum(0)
    se = f.std(0, ddof=1) * math.sqrt(B) / tot.max()
    assert np.all(film.cpu().numpy()[:, 0] == 0.0)             # fluorescence only
    return spd.cpu().numpy().astype(np.float64), f, se


def _bound():
    lam = cf.grid_lambda(101)
    sa = cf.dye_sigma_a(lam, [(550, 20, 1)], 7e4, CONC, 101)
    return 1.0 - math.exp(-sa.max() * 2 * 0.3)


def test_fluorescent_spd_follows_emission_spectrum():
    spd, f, se = _gpu_spd(550.0, 1 << 26, seed=1)
    # against the oracle's reduction of its own film
    scene = workloads.validation_scene(lambda_x=550.0, conc_uM=CONC, sigma_s=SIGMA_S)
    o = oracle.render(scene, workloads.make_run(1 << 24, seed=2, parity_batches=B,
                                                fluorescence_only=True))["film"]
    of = o[:, 1].sum((1, 2))
    z = batch_z(f, of)
    assert z.size >= 25   # the emission band: 580 +- 3 sd nm at 5 nm
    check_z(z, "fluorescent SPD: GPU vs oracle", dof=B - 1)
    # against the dye's emission spectrum
    pmf = cf.emission_pmf(101, [(580, 25, 1)])
    pmf_n = pmf / pmf.max()
    m = pmf_n > 0.1
    dev = np.abs(spd - pmf_n)[m]
    assert np.all(dev <= _bound() + 4 * se[m]), (dev.max(), _bound())
    assert abs(int(np.argmax(spd)) - int(np.argmax(pmf))) <= 1


def test_spd_shape_independent_of_excitation():
    a, _, sa = _gpu_spd(540.0, 1 << 26, seed=3)
    b, _, sb = _gpu_spd(565.0, 1 << 26, seed=4)
    m = (a > 0.1) | (b > 0.1)
    dev = np.abs(a - b)[m]
    assert np.all(dev <= _bound() + 4 * np.hypot(sa, sb)[m]), dev.max()
