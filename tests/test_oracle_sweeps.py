"""The experiment sweeps' scenes on the oracle: non-scattering dye slabs,
whose fluorescent escape spectra have a 1-D quadrature form (first-collision
law, the dye's share of sigma_t, QY, the emission PMF of eq. 10, uncollided
escape), across excitation wavelength and concentration."""
from __future__ import annotations

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from stats import check_z, multinomial_z

N = 101


def slab_closed_form(lambda_x, conc_uM, d=1.0, bg=0.01):
    lam = cf.grid_lambda(N)
    k = int(round((lambda_x - 300.0) / 5.0))
    dye = workloads.SWEEP_DYE
    sa = cf.dye_sigma_a(lam, [(*dye["abs"], 1.0)], dye["epsilon"], conc_uM, N)
    st = bg + sa
    pmf = cf.emission_pmf(N, [(*dye["em"], 1.0)])
    return cf.dye_slab_fluorescent_film(d, st[k], sa[k], dye["qy"], pmf, st)


def sweep_z(films, n, cases):
    z = []
    for f, (lx, c) in zip(films, cases):
        R, T = slab_closed_form(lx, c)
        if (R.sum() + T.sum()) * n < 20:
            assert f[1].sum() * n < 20 + 5 * np.sqrt(20)
            continue
        z.append(multinomial_z(f[1, 0], n, R))
        z.append(multinomial_z(f[1, 1], n, T))
    return np.concatenate(z)


@pytest.mark.parametrize("sweep", ["excitation", "concentration"])
def test_oracle_sweep_instances_match_closed_form(sweep):
    n = 1 << 16
    if sweep == "excitation":
        lams = [400.0, 450.0, 490.0, 530.0, 600.0]
        scenes, runs = workloads.excitation_scan(lams, paths=n)
        cases = [(lx, 10.0) for lx in lams]
    else:
        concs = [0.1, 10.0, 1000.0]
        scenes, runs = workloads.concentration_sweep(concs, paths=n)
        cases = [(490.0, c) for c in concs]
    films = [oracle.render(s, r)["film"][0] for s, r in zip(scenes, runs)]
    check_z(sweep_z(films, n, cases), f"oracle {sweep} sweep vs closed form")
