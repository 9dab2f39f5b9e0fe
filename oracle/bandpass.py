"""Oracle: ArPLS bandpass normalisation (Sec. 3.1; parameters lam, ratio and
itermax of Sec. 4.5) and the non-centred cross-correlation matrix of the
bandpass-subtracted power.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3.1: the samples of each channel are aggregated over a time interval, the
bandpass shape across channels is fitted by ArPLS (asymmetrically reweighted
penalised least squares, Baek et al. 2015), and the fitted bandpass is
subtracted from every time sample of the channel. Readings:

* the aggregation interval is the sub-interval of the CCM, so the bandpass of
  beam b in sub-interval k is y_j = S_b(k, j) / L over the channels j (the
  channel means, exactly the sums of Eq. 1 divided by L);
* ArPLS as published: with D the second-difference operator and H = lam D^T D,
  start from w = 1; solve (W + H) z = W y; d = y - z; m, s = mean and sample
  standard deviation (ddof 1) of the negative residuals; new weights
  w_t = 1 / (1 + exp(2 (d - (2 s - m)) / s)); stop when ||w - w_t|| / ||w|| <
  ratio (the fit of that pass is kept) or after itermax passes; the baseline
  is the last z;
* non-centred CCM: <B'_a B'_b> = (1/L) sum_t (x_a(t) - z_a)(x_b(t) - z_b) with
  x' the bandpass-subtracted power and z the cell's baseline values: the raw
  second moment of x', the reading C1 of the paper's <B_a B_b> taken without
  centring or normalisation. It follows from the exact sums:
      M_ab = (S_ab - z_b S_a - z_a S_b + L z_a z_b) / L.
"""
from __future__ import annotations

import math

import numpy as np


def second_difference(F: int) -> np.ndarray:
    """D [(F - 2), F]: (D z)_i = z_i - 2 z_{i+1} + z_{i+2}."""
    D = np.zeros((max(F - 2, 0), F))
    for i in range(F - 2):
        D[i, i], D[i, i + 1], D[i, i + 2] = 1.0, -2.0, 1.0
    return D


def arpls(y: np.ndarray, lam: float = 1e5, ratio: float = 0.05, itermax: int = 100):
    """ArPLS baseline of one spectrum y [F] (Baek et al. 2015), dense FP64
    solves (small F only). Returns (z [F], passes)."""
    y = np.asarray(y, dtype=np.float64)
    F = y.size
    if F < 3:
        return y.copy(), 0
    D = second_difference(F)
    H = lam * (D.T @ D)
    w = np.ones(F)
    z = y.copy()
    passes = 0
    for _ in range(itermax):
        passes += 1
        z = np.linalg.solve(np.diag(w) + H, w * y)
        d = y - z
        dn = d[d < 0]
        if dn.size < 2:
            break
        m = dn.mean()
        s = dn.std(ddof=1)
        if not (s > 0):
            break
        with np.errstate(over="ignore"):           # exp overflow: weight 0, as intended
            wt = 1.0 / (1.0 + np.exp(2.0 * (d - (2.0 * s - m)) / s))
        if np.linalg.norm(w - wt) / np.linalg.norm(w) < ratio:
            break
        w = wt
    return z, passes


def bandpass_from_sums(S: np.ndarray, L, lam=1e5, ratio=0.05, itermax=100):
    """Baselines of every (sub-interval, beam) from the sums S [nsub, nchan,
    nbeam] and samples per sub-interval L (scalar or [nsub]): returns z
    [nsub, nchan, nbeam] and the pass counts [nsub, nbeam]."""
    S = np.asarray(S, dtype=np.float64)
    nsub, nchan, nbeam = S.shape
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (nsub,))
    z = np.zeros_like(S)
    passes = np.zeros((nsub, nbeam), dtype=np.int64)
    for k in range(nsub):
        for b in range(nbeam):
            z[k, :, b], passes[k, b] = arpls(S[k, :, b] / Ls[k], lam, ratio, itermax)
    return z, passes


def noncentred_ccm(S: np.ndarray, S2: np.ndarray, L, z: np.ndarray) -> np.ndarray:
    """M_ab = (S_ab - z_b S_a - z_a S_b + L z_a z_b) / L per cell: the raw
    second-moment matrix of the bandpass-subtracted samples (FP64).
    S [..., n], S2 [..., n, n], z [..., n] (0 for no bandpass)."""
    S = np.asarray(S, dtype=np.float64)
    S2 = np.asarray(S2, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    Lf = np.asarray(L, dtype=np.float64)
    Lb = Lf[..., None, None] if Lf.ndim else Lf
    za, zb = z[..., :, None], z[..., None, :]
    Sa, Sb = S[..., :, None], S[..., None, :]
    return (S2 - zb * Sa - za * Sb + Lb * za * zb) / Lb


def statistic_general(M: np.ndarray):
    """s = lambda_1^2 / sum lambda^2 for symmetric matrices M [..., n, n]
    (Sec. 3.3; the eigenvalue of largest magnitude), with sum lambda^2 =
    ||M||_F^2. Returns (s, lambda_1)."""
    w = np.linalg.eigvalsh(M)
    idx = np.argmax(np.abs(w), axis=-1)
    lam1 = np.take_along_axis(w, idx[..., None], axis=-1)[..., 0]
    f2 = (M * M).sum(axis=(-1, -2))
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(f2 > 0, lam1 * lam1 / f2, 0.0)
    return s, lam1
