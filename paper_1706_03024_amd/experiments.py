"""The paper's experiments (sec. 5) as batched sweeps, and the reduction its
figures report: the fluorescent spectral power distribution (SPD),
peak-normalised.

A sweep is a list of escape-sensor instances rendered by one persistent
launch (fpt_batch_*).  For camera films the SPD is averaged over the pixels
that receive fluorescence before normalisation.  All work is on the device.
"""
from __future__ import annotations

import torch

from .renderer import Batch, new_tallies


def run_sweep(scenes, runs, tune=None, tallies=False):
    """Renders every instance of a sweep in one batched launch; returns the
    escape films [n][2 comp][2 side][n_bins] (fractions of source photons)
    and, if asked, the per-instance tallies."""
    b = Batch(scenes, runs, tune=tune)
    try:
        films = b.new_films()
        t = new_tallies(len(scenes)) if tallies else None
        b.render(films, t)
        torch.cuda.current_stream().synchronize()
    finally:
        b.close()
    return (films, t) if tallies else films


def fluorescent_spd(films):
    """Escape films [n][2][2][N] -> fluorescent SPD [n][N]: component 1
    (emitted at least once), reflected plus transmitted."""
    return films[:, 1, 0, :] + films[:, 1, 1, :]


def pinhole_spd(film):
    """Camera film [B][2][H][W][N] -> fluorescent SPD [N]: component 1 summed
    over parity batches, averaged over the pixels that receive any."""
    f = film[:, 1].sum(0)                      # [H][W][N]
    lit = f.sum(-1) > 0
    n = int(lit.sum().item())
    if n == 0:
        return torch.zeros(f.shape[-1], dtype=f.dtype, device=f.device)
    return f[lit].sum(0) / n


def rebin(film, factor):
    """Sums a fine spectral axis (last) onto a grid `factor` times coarser with
    the same end points: coarse point k collects the fine points within half a
    coarse spacing of it, a point on a boundary shared by two coarse points
    going half to each (so the total is kept).  For a 1-nm grid of 300-800 nm
    (501 points) and factor 5 this gives the 101-point grid."""
    n = film.shape[-1]
    if (n - 1) % factor:
        raise ValueError("the fine grid does not refine the coarse one")
    m = (n - 1) // factor + 1
    # distance of fine point j from coarse point k, in fine steps
    dist = (torch.arange(n, device=film.device)[:, None] * 2
            - torch.arange(m, device=film.device)[None, :] * (2 * factor)).abs()
    one, half = torch.ones((), dtype=film.dtype, device=film.device), torch.tensor(0.5, dtype=film.dtype,
                                                                                   device=film.device)
    w = torch.where(dist < factor, one, torch.where(dist == factor, half, torch.zeros_like(one)))
    return film @ w


def normalized(spd):
    """Each spectrum divided by its peak (all-zero spectra stay zero)."""
    peak = spd.amax(-1, keepdim=True)
    return torch.where(peak > 0, spd / torch.where(peak > 0, peak, torch.ones_like(peak)),
                       torch.zeros_like(spd))
