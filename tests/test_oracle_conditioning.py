"""Pins of the oracle's conditioning probe (oracle.replay_condition), which
sets how far a replayed fp32 path may drift from the fp64 walk.

* Switched off (eta = 0) the walk is the plain walk, record for record.
* Beer-Lambert slab (T1 without scattering), a normal beam: a path absorbed at depth z has its
  one computed position (0, 0, z) scaled by 1 +- eta, so its position
  condition number is exactly z / max(z, scale); a path that escapes through
  a face lies exactly on that face's plane (set, not computed) and the beam
  axis, so it is 0.  The direction is the beam's, given, never computed: 0.
* First order: halving eta leaves the condition numbers of well-conditioned
  paths unchanged (the probe measures a derivative, not a large deviation).
"""
from __future__ import annotations

import numpy as np

import oracle
import workloads


def test_probe_off_is_the_plain_walk():
    scene, run = workloads.cornell_config()
    sub = dict(run, path_count=512)
    a = oracle.render(scene, sub, records=True)["records"]
    b = oracle.render(scene, dict(sub, perturb_eta=0.0, perturb_pattern=7), records=True)["records"]
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_beer_lambert_condition_numbers():
    scene = workloads.t1_beer_lambert(sigma_s=0.0, sigma_a=1.0)
    run = workloads.make_run(1 << 12, seed=3)
    c = oracle.replay_condition(scene, run, scale=1.0)
    rec = c["records"]
    assert not c["unstable"].any()
    esc = rec["exit_code"] <= 1
    bg = rec["exit_code"] == 2
    assert esc.sum() > 100 and bg.sum() > 100 and np.all(esc | bg)
    assert np.all(c["kappa_pos"][esc] == 0.0)
    z = rec["pos"][bg, 2]
    np.testing.assert_allclose(c["kappa_pos"][bg], z / np.maximum(z, 1.0), rtol=1e-6)
    assert np.all(c["kappa_dir"] == 0.0)


def test_first_order():
    scene, run = workloads.cornell_config()
    sub = dict(run, path_begin=1000, path_count=1024)
    a = oracle.replay_condition(scene, sub, eta=2.0 ** -23)
    b = oracle.replay_condition(scene, sub, eta=2.0 ** -24)
    ok = ~(a["unstable"] | b["unstable"])
    for k in ("kappa_pos", "kappa_splat"):
        x, y = a[k][ok], b[k][ok]
        m = (x > 0) & (x < 1e3)
        assert m.sum() > 100
        r = y[m] / x[m]
        assert np.median(np.abs(r - 1.0)) < 0.05, (k, np.quantile(r, [0.1, 0.5, 0.9]))
