"""Per-path replay comparison of GPU records with oracle records.

Both sides draw identical Philox streams, so every path makes the same
decisions except where a decision is within rounding of its threshold.  The
oracle logs each path's smallest relative decision margin; paths below
`margin` are "marginal" and excluded (their count is reported and bounded).
Integer fields must match exactly on the rest, and fp32 state within
`rtol` * max(|a|, |b|, scale).
"""
from __future__ import annotations

import numpy as np


def compare_records(gpu, orc, scale=1.0, rtol=1e-5, margin=1e-5, max_marginal_frac=0.001,
                    check_splat=True, splat_rtol=1e-4):
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
    for f in ("pos", "dir"):
        a = gpu[f][ok].astype(np.float64)
        b = orc[f][ok]
        fin = np.isfinite(b)
        tol = rtol * np.maximum(np.maximum(np.abs(a), np.abs(b)), scale)
        err = np.abs(a - b)
        bad = fin & (err > tol)
        assert not bad.any(), (f, report, np.nonzero(bad.any(1))[0][:5], float(err[fin].max()))
    if check_splat:
        a = gpu["splat_sum"][ok].astype(np.float64)
        b = orc["splat_sum"][ok]
        tol = splat_rtol * np.maximum(np.abs(b), 1e-30) + 1e-30
        bad = np.abs(a - b) > tol
        assert not bad.any(), ("splat_sum", report, np.nonzero(bad)[0][:5])
    report["max_pos_err"] = float(np.max(np.abs(gpu["pos"][ok] - orc["pos"][ok]),
                                         initial=0.0, where=np.isfinite(orc["pos"][ok])))
    return report
