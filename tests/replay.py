"""Per-path replay comparison of GPU records with oracle records.

Both sides draw identical Philox streams, so every path makes the same
decisions and passes through the same states, up to rounding.  The bar is a
relative error of 1e-5 per path, made precise as follows.

* Marginal paths.  The oracle logs each path's smallest relative decision
  margin (a uniform against its threshold, a flight length against the
  distance to the next surface, ...).  Paths with a margin below `margin`
  (2e-6, about 30 fp32 ulps) or whose integer outcome changes when the
  oracle perturbs its own state by one fp32 ulp (`unstable`) are excluded;
  their share is bounded.
* Integer outcomes (vertex count, scatters, emissions, exit code, wavelength
  bin, component) are exactly equal on every other path.
* Floating-point fields (exit position and direction, the path's deposited
  film total, its gradient contribution) are within rtol = 1e-5 relative,
  scaled by the path's condition number kappa >= 1:
        |gpu - oracle| <= 1e-5 * max(1, kappa) * max(|gpu|, |oracle|, floor).
  kappa comes from the oracle alone (oracle.replay_condition): the change of
  the field when every position, direction and accumulator the oracle
  computes is perturbed by one fp32 ulp, divided by that ulp.  A path with
  kappa <= 1 is held to plain 1e-5; a path that amplifies rounding -- grazing
  wall bounces multiply a position error by about 1/|cos| each, and a deposit
  through optical depth tau has relative sensitivity tau to its chord -- is
  held to a relative error of 1e-5 in every vertex state, the same bar
  expressed where the walk makes its rounding.  No share of paths is exempt.
  Floors: positions against the scene scale, directions against 1, deposits
  and gradients against 2^-100 (far below any value that reaches a film; fp32
  intermediates of such values -- a transmittance near 2^-126 times geometry
  factors -- lose significant bits in the subnormal range).
* The report also gives how many paths exceed plain 1e-5 and the GPU's error
  in units of kappa * ulp (the effective fp32 rounding per vertex), whose
  median and 99th percentile are bounded: a systematic GPU inaccuracy shows
  there even on well-conditioned paths.
"""
from __future__ import annotations

import numpy as np

import oracle

ULP = 2.0 ** -23
TINY = 2.0 ** -100


def oracle_replay(scene, run, max_vertices=0, grad_film=None, camera=False, scale=1.0):
    """Oracle records of a path range with their condition numbers."""
    return oracle.replay_condition(scene, run, max_vertices=max_vertices, grad_film=grad_film,
                                   camera=camera, scale=scale)


def _check(label, err, kappa, rtol, report, ulp_q50, ulp_q99):
    tol = rtol * np.maximum(1.0, kappa)
    bad = np.nonzero(err > tol)[0]
    report[label + "_over_1e-5"] = int(np.sum(err > rtol))
    report[label + "_kappa_gt_1"] = int(np.sum(kappa > 1.0))
    ratio = err / np.maximum(kappa * ULP, ULP)
    if ratio.size:
        report[label + "_ulps_q50"] = float(np.quantile(ratio, 0.5))
        report[label + "_ulps_q99"] = float(np.quantile(ratio, 0.99))
    assert bad.size == 0, (label, report, bad[:5], err[bad[:5]], kappa[bad[:5]])
    if ratio.size:
        assert report[label + "_ulps_q50"] <= ulp_q50 and report[label + "_ulps_q99"] <= ulp_q99, \
            (label, report)


def compare_records(gpu, cond, scale=1.0, rtol=1e-5, margin=2e-6, max_marginal_frac=0.001,
                    check_splat=True, gpu_grad=None, ulp_q50=4.0, ulp_q99=32.0):
    """Compare GPU records (and per-path gradients) with an oracle_replay() result."""
    orc = cond["records"]
    assert len(gpu) == len(orc)
    marginal = (orc["margin"] < margin) | cond["unstable"]
    ok = ~marginal
    n_marg = int(marginal.sum())
    report = {"paths": len(orc), "marginal": n_marg}
    assert n_marg <= max(2, max_marginal_frac * len(orc)), report
    for f in oracle.INT_FIELDS:
        a = gpu[f][ok].astype(np.int64)
        b = orc[f][ok].astype(np.int64)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (f, report, bad[:5], a[bad[:5]], b[bad[:5]],
                               orc["margin"][ok][bad[:5]])
    for f, floor in (("pos", scale), ("dir", 1.0)):
        a = gpu[f][ok].astype(np.float64)
        b = orc[f][ok]
        fin = np.all(np.isfinite(b), 1)
        err = (np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)).max(1)
        _check(f, err[fin], cond["kappa_" + f][ok][fin], rtol, report, ulp_q50, ulp_q99)
    if check_splat:
        a = gpu["splat_sum"][ok].astype(np.float64)
        b = orc["splat_sum"][ok]
        err = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), TINY)
        _check("splat", err, cond["kappa_splat"][ok], rtol, report, ulp_q50, ulp_q99)
    if gpu_grad is not None:
        a = np.asarray(gpu_grad, np.float64)[ok]
        b = cond["record_grad"][ok]
        err = np.linalg.norm(a - b, axis=1) / np.maximum(
            np.maximum(np.linalg.norm(a, axis=1), np.linalg.norm(b, axis=1)), TINY)
        _check("grad", err, cond["kappa_grad"][ok], rtol, report, ulp_q50, ulp_q99)
    return report


def check_grad_total(total, gpu_grad, cond, rtol=1e-5, margin=2e-6):
    """A reduced gradient (fpt_render_adjoint over the same paths) against the
    per-path contributions of the records launch and of the oracle.  The
    adjoint launch walks long paths in wave-cooperative rounds (positions by
    prefix sums), the records launch one vertex at a time, so the two are two
    fp32 walks of each path: the total may differ from either sum by
    rtol * max(1, kappa) of each path's contribution, all of a marginal path's
    (it may decide otherwise), and the fp32 rounding of the partial sums.
    Returns the largest deviation of each comparison over its allowance."""
    total = np.asarray(total, np.float64)
    rg = np.asarray(gpu_grad, np.float64)
    og = cond["record_grad"]
    marginal = (cond["records"]["margin"] < margin) | cond["unstable"]
    k = np.maximum(1.0, cond["kappa_grad"])[:, None]
    mag = np.abs(og) + np.abs(rg)
    allow = (rtol * k * mag)[~marginal].sum(0) + mag[marginal].sum(0) + 2.0 ** -20 * mag.sum(0)
    d_self = np.abs(total - rg.sum(0))
    d_orc = np.abs(total - og.sum(0))
    assert np.all(d_self <= allow + TINY), (d_self, allow)
    assert np.all(d_orc <= allow + TINY), (d_orc, allow)
    return (float(np.max(d_self / np.maximum(allow, TINY))),
            float(np.max(d_orc / np.maximum(allow, TINY))))
