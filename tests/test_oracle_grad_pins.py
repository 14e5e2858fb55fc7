"""Pins of the oracle's path-replay gradient estimator (likelihood-ratio form:
d E[v] = E[v d log p(path) + d v]) against closed-form derivatives and against
central finite differences of the forward walk with common random numbers."""
from __future__ import annotations

import math

import numpy as np

import closed_forms as cf
import oracle
import workloads
from stats import check_z


def _fl_T_total(conc, qy, lx=490.0, d=1.0, bg=0.05):
    N = 101
    lam = cf.grid_lambda(N)
    k = int(round((lx - 300) / 5))
    sa = cf.dye_sigma_a(lam, [(490, 20, 1)], 7e4, conc, N)
    st = bg + sa
    pmf = cf.emission_pmf(N, [(520, 25, 1)])
    R, T = cf.dye_slab_fluorescent_film(d, st[k], sa[k], qy, pmf, st)
    return T.sum() + R.sum()


def test_dye_slab_gradients_match_closed_form():
    """Non-scattering dye slab: d/dc and d/dQY of the total fluorescent escape
    (closed form, differentiated in fp64) equal the gradient estimator's mean.
    Parameter order: [conc(medium 0, dye 0), QY(dye 0), sigma_s(medium 0)]."""
    conc, qy = 20.0, 0.8
    s = workloads.t6_dye_slab(conc_uM=conc, qy=qy)
    n = 1 << 17
    g = np.zeros(oracle.film_shape(s))
    g[0, 1] = 1.0  # fluorescent component, both faces, all bins
    o = oracle.render(s, workloads.make_run(n, seed=61), grad_film=g, record_grad=True)
    pg = o["record_grad"] * n  # per-path contributions, mean = gradient
    mean = pg.mean(0)
    se = pg.std(0, ddof=1) / math.sqrt(n)
    h = 1e-4
    d_c = (_fl_T_total(conc * (1 + h), qy) - _fl_T_total(conc * (1 - h), qy)) / (2 * h * conc)
    d_q = (_fl_T_total(conc, qy * (1 + h)) - _fl_T_total(conc, qy * (1 - h))) / (2 * h * qy)
    assert np.allclose(o["grad"], mean, rtol=1e-9, atol=0)
    z = [(mean[0] - d_c) / se[0], (mean[1] - d_q) / se[1]]
    check_z(z, "dye slab d/dc, d/dQY")
    # the ballistic elastic transmission of a non-scattering slab: d/dc T = -kappa d T
    g2 = np.zeros(oracle.film_shape(s))
    g2[0, 0, 1, 38] = 1.0
    o2 = oracle.render(s, workloads.make_run(n, seed=62), grad_film=g2, record_grad=True)
    pg2 = o2["record_grad"][:, 0] * n
    kappa = cf.dye_sigma_a(cf.grid_lambda(101)[38], [(490, 20, 1)], 7e4, 1.0, 101)
    st = 0.05 + kappa * conc
    expect = -kappa * 1.0 * math.exp(-st * 1.0)
    assert abs(pg2.mean() - expect) < 4.5 * pg2.std(ddof=1) / math.sqrt(n)


def _fd(scene_fn, theta, i, h, run, g):
    tp = list(theta)
    tm = list(theta)
    tp[i] *= 1 + h
    tm[i] *= 1 - h
    fp = oracle.render(scene_fn(tp), run)["film"]
    fm = oracle.render(scene_fn(tm), run)["film"]
    B = fp.shape[0]
    # per-batch linear functional (each batch is an independent estimate)
    vals = ((fp - fm) * g).reshape(B, -1).sum(1) / (2 * h * theta[i])
    return vals


def test_camera_gradients_match_finite_differences():
    """Small Cornell scene: the gradient of a fixed linear functional <g, I>
    w.r.t. concentration, QY and sigma_s of each sphere agrees with central
    differences of the forward walk using common random numbers."""
    W = 12
    B = 32
    rng = np.random.default_rng(5)

    def scene_fn(theta):
        s = workloads.cornell_scene(W, W)
        for m in range(3):
            s["media"][m]["dyes"][0][1] = theta[m]
            s["dyes"][m]["qy"] = theta[3 + m]
            s["media"][m]["sigma_s"] = theta[6 + m]
        # brighter dyes so the fluorescent component is not negligible
        return s

    base = workloads.cornell_scene(W, W)
    theta = [base["media"][m]["dyes"][0][1] * 20 for m in range(3)] + \
            [base["dyes"][m]["qy"] for m in range(3)] + \
            [base["media"][m]["sigma_s"] / 10 for m in range(3)]
    theta[5] = 0.6
    s = scene_fn(theta)
    n = 1 << 18
    run = workloads.make_run(n, seed=7, parity_batches=B)
    g = 1.0 + rng.random(oracle.film_shape(s, B)[1:])  # positive: a weighted brightness
    g = np.broadcast_to(g, oracle.film_shape(s, B)).copy()
    o = oracle.render(s, run, grad_film=g / B, record_grad=True)
    pg = o["record_grad"]
    # batch means of the estimator: path p belongs to batch p % B
    per_batch = np.stack([pg[b::B].sum(0) for b in range(B)])
    z = []
    resolved = 0
    for i in range(9):
        fd = _fd(scene_fn, theta, i, 0.02, run, g)
        est = per_batch[:, i] * B
        se_est = math.sqrt(est.var(ddof=1) / B)
        se = math.sqrt(est.var(ddof=1) / B + fd.var(ddof=1) / B)
        resolved += abs(est.mean()) > 3 * se_est
        z.append((est.mean() - fd.mean()) / se)
    assert resolved >= 5, "the functional's gradient is not resolved: the check would be vacuous"
    check_z(z, "camera gradient vs central differences", dof=B - 1)
