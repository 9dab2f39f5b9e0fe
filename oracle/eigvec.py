"""Oracle: per-beam eigenvector threshold (Sec. 3.3 last paragraph; Sec. 4.5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

After the eigenvalue mask is built, the elements of each flagged cell's
dominant eigenvector decide which beams carry the interference: a beam whose
element magnitude exceeds its threshold is masked in that cell. Each beam's
threshold is set from a Gaussian fit to that beam's eigenvector elements over
the cells that are not flagged (Fig. 3), at kappa_v standard deviations
(kappa_v = 1 for the FAST data, Sec. 4.5).

Readings: the fitted quantity is |q_1b| (the test is on magnitudes); the fit
is the moment fit (mean, population standard deviation) over eligible,
unflagged cells; a single pass, no iteration; strict '>'.
"""
from __future__ import annotations

import numpy as np


def eigvec_mask(v1: np.ndarray, mask: np.ndarray, eligible: np.ndarray,
                kappa_v: float = 1.0):
    """Per-beam mask.

    v1: [..., nbeam] dominant eigenvectors per cell; mask, eligible: [...]
    bool. Returns (beam_mask [nbeam, ...] bool, mu [nbeam], sigma [nbeam]).
    """
    v1 = np.asarray(v1, dtype=np.float64)
    a = np.abs(v1)
    clean = np.asarray(eligible, bool) & ~np.asarray(mask, bool)
    nbeam = v1.shape[-1]
    mu = np.full(nbeam, np.nan)
    sd = np.full(nbeam, np.nan)
    out = np.zeros((nbeam,) + mask.shape, dtype=bool)
    for b in range(nbeam):
        vals = a[..., b][clean]
        if vals.size == 0:
            continue
        mu[b] = vals.mean()
        sd[b] = np.sqrt(np.mean((vals - mu[b]) ** 2))
        out[b] = np.asarray(mask, bool) & (a[..., b] > mu[b] + kappa_v * sd[b])
    return out, mu, sd
