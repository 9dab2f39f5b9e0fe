"""Oracle: the whole per-block path, composed from the other oracle modules.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For every cell (sub-interval k, channel j) of a block: exact sums (Eq. 1),
FP64 Pearson correlation, eigendecomposition (Eq. 2), statistic
lambda_1^2 / sum lambda^2 (Sec. 3.3); then one iterative clip over all cells
(Sec. 3.3, Sec. 4.5) and optionally the per-beam eigenvector stage.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import ccm, clip, eig, eigvec

STATUS_DEGENERATE = 1
STATUS_PROTECTED = 4


@dataclass
class CellResult:
    S: np.ndarray        # [nsub, nchan, nbeam] int64
    S2: np.ndarray       # [nsub, nchan, nbeam, nbeam] int64
    r: np.ndarray        # [nsub, nchan, nbeam, nbeam] float64
    w: np.ndarray        # [nsub, nchan, nbeam] float64, |lambda| descending
    v1: np.ndarray       # [nsub, nchan, nbeam] float64
    frob2: np.ndarray    # [nsub, nchan]
    stat: np.ndarray     # [nsub, nchan]
    degenerate: np.ndarray  # [nsub, nchan] bool


def cells(x: np.ndarray, L: int, nsub: int, t0: int = 0, sums: str = "fp64") -> CellResult:
    """Per-cell part of the path for x[beam, time, channel] uint8."""
    if sums == "fp64":
        S, S2 = ccm.sums_fp64(x, L, nsub, t0)
    elif sums == "int64":
        S, S2 = ccm.sums_int64(x, L, nsub, t0)
    else:
        S, S2 = ccm.sums_loops(x, L, nsub, t0)
    r, deg = ccm.correlation(S, S2, L)
    f2 = ccm.frobenius2(r)
    w, v1 = eig.cell_eigen(r)
    s = eig.statistic(w[..., 0], f2)
    return CellResult(S, S2, r, w, v1, f2, s, deg)


def eligible_cells(degenerate: np.ndarray, protect_chan=None) -> np.ndarray:
    """Cells that enter the fit and may be flagged: not degenerate and not in
    a preserved channel (Sec. 4.3)."""
    ok = ~np.asarray(degenerate, bool)
    if protect_chan is not None:
        ok = ok & ~np.asarray(protect_chan, bool)[None, :]
    return ok


def block(x: np.ndarray, L: int, nsub: int, kappa: float = 3.0, max_iter: int = 50,
          protect_chan=None, kappa_v: float | None = None, t0: int = 0):
    """Whole path for one block; returns (CellResult, ClipResult, beam_mask or None)."""
    cr = cells(x, L, nsub, t0)
    ok = eligible_cells(cr.degenerate, protect_chan)
    res = clip.clip_iterative(cr.stat, ok, kappa, max_iter)
    bm = None
    if kappa_v is not None:
        bm, _, _ = eigvec.eigvec_mask(cr.v1, res.mask, ok, kappa_v)
    return cr, res, bm
