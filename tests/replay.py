"""Per-path replay comparison of GPU records with oracle records.

Both sides draw identical Philox streams, so every path makes the same
decisions except where a decision lies within rounding of its threshold.  The
oracle logs each path's smallest relative decision margin; paths below
`margin` (2e-6, about 30 fp32 ulps) are "marginal" and excluded; their share
is bounded.

Acceptance on the remaining paths:
  * integer outcomes (vertex count, scatters, emissions, exit, wavelength bin,
    component) exactly equal;
  * exit position and direction within `rtol` = 1e-5 relative (floor: the
    scene scale) for at least `frac_ok` of the paths, and within 1e-3 for all:
    fp32 position rounding grows along long walks, and grazing wall bounces
    amplify it by 1/|cos| per bounce (billiard divergence), so a small tail
    drifts past 1e-5 without any decision changing;
  * the path's deposited film total within `splat_rtol` relative for at least
    `frac_ok` of the paths: a splat's transmittance exp(-sigma_t l) turns a
    position difference dx into a relative change sigma_t dx, so in media with
    sigma_t ~ 1e2-1e3 /mm the tolerance is 1e-5 * max(1, sigma_t,max * scale).
    With `splat_floor` > 0, deposits below it are compared in absolute terms
    against it: a deposit made only through deep connections (transmittance
    1e-4 and below) has relative sensitivity sigma_t * L * (dx / L), large for
    large optical depth, while its share of any film cell stays negligible.
"""
from __future__ import annotations

import numpy as np


def compare_records(gpu, orc, scale=1.0, rtol=1e-5, margin=2e-6, max_marginal_frac=0.001,
                    check_splat=True, sigma_t_max=1.0, frac_ok=0.995, splat_floor=0.0):
    assert len(gpu) == len(orc)
    marginal = orc["margin"] < margin
    ok = ~marginal
    n_marg = int(marginal.sum())
    report = {"paths": len(orc), "marginal": n_marg}
    assert n_marg <= max(2, max_marginal_frac * len(orc)), report
    for f in ("n_vertices", "n_scatter", "n_emit", "exit_code", "lambda", "comp"):
        a = gpu[f][ok].astype(np.int64)
        b = orc[f][ok].astype(np.int64)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (f, report, bad[:5], a[bad[:5]], b[bad[:5]],
                               orc["margin"][ok][bad[:5]])
    worst = 0.0
    for f in ("pos", "dir"):
        a = gpu[f][ok].astype(np.float64)
        b = orc[f][ok]
        fin = np.all(np.isfinite(b), 1)
        rel = (np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), scale)).max(1)[fin]
        frac = float(np.mean(rel <= rtol)) if rel.size else 1.0
        report[f + "_frac_1e-5"] = frac
        worst = max(worst, float(rel.max(initial=0.0)))
        assert frac >= frac_ok and rel.max(initial=0.0) <= 1e-3, (f, report, float(rel.max()))
    report["pos_worst"] = worst
    if check_splat:
        a = gpu["splat_sum"][ok].astype(np.float64)
        b = orc["splat_sum"][ok]
        tol = rtol * max(1.0, sigma_t_max * scale)
        rel = np.abs(a - b) / np.maximum(np.abs(b), max(1e-30, splat_floor))
        rel = rel[(a != 0) | (b != 0)]
        frac = float(np.mean(rel <= tol)) if rel.size else 1.0
        report["splat_frac"] = frac
        assert frac >= frac_ok and rel.max(initial=0.0) <= 1e-2, ("splat_sum", report,
                                                                   float(rel.max()))
    return report
