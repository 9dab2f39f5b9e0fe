"""Oracle: exact per-cell sums and the cross-correlation matrix (Sec. 3.2, Eq. 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A cell is one (sub-interval k, frequency channel j). Its CCM has one entry per
pair of beams (a, b): the correlation over the cell's time samples of the total
power recorded by the two beams (Sec. 3.2, Eq. 1). The number of samples in a
cell is N_s = T_k / t_s (Sec. 3.2); here it is given directly as an integer L.

Reading of the entry <B_a B_b>: the Pearson correlation over the L samples of
the cell (the paper calls C a correlation matrix and interprets normalised
eigenvalues as shares of variance, Sec. 3.2-3.3). It is computed exactly:

    S_a  = sum_t x_a(t)                         (integer)
    S_ab = sum_t x_a(t) x_b(t)                  (integer)
    N_ab = L * S_ab - S_a * S_b                 (integer, = L^2 * covariance)
    r_ab = N_ab / sqrt(N_aa * N_bb)             (FP64),  r_aa = 1

A beam with N_aa = 0 (constant power in the cell) has no defined correlation;
its off-diagonal entries are set to 0 and the cell is marked degenerate.

Input layout used throughout the oracle: ``x[beam, time, channel]`` uint8.
"""
from __future__ import annotations

import numpy as np


def cell_slices(x: np.ndarray, L: int, nsub: int, t0: int = 0):
    """Return x reshaped to [nbeam, nsub, L, nchan] for sub-intervals
    [t0 + kL, t0 + (k+1)L), k < nsub (Sec. 3.2: a sub-interval holds N_s
    consecutive samples)."""
    nbeam, nsamp, nchan = x.shape
    if t0 + nsub * L > nsamp:
        raise ValueError("sub-intervals run past the end of the data")
    return x[:, t0:t0 + nsub * L, :].reshape(nbeam, nsub, L, nchan)


def sums_loops(x: np.ndarray, L: int, nsub: int, t0: int = 0):
    """Eq. 1 sums by plain Python loops (tiny inputs only).

    Returns (S [nsub, nchan, nbeam], S2 [nsub, nchan, nbeam, nbeam]) as
    Python-int-valued int64 arrays.
    """
    nbeam, _, nchan = x.shape
    S = np.zeros((nsub, nchan, nbeam), dtype=np.int64)
    S2 = np.zeros((nsub, nchan, nbeam, nbeam), dtype=np.int64)
    for k in range(nsub):
        for j in range(nchan):
            for a in range(nbeam):
                sa = 0
                for t in range(t0 + k * L, t0 + (k + 1) * L):
                    sa += int(x[a, t, j])
                S[k, j, a] = sa
                for b in range(nbeam):
                    sab = 0
                    for t in range(t0 + k * L, t0 + (k + 1) * L):
                        sab += int(x[a, t, j]) * int(x[b, t, j])
                    S2[k, j, a, b] = sab
    return S, S2


def sums_int64(x: np.ndarray, L: int, nsub: int, t0: int = 0):
    """Eq. 1 sums in exact int64 arithmetic (vectorised over cells).

    Exact while L * 255^2 < 2^63, i.e. for any L that fits in memory.
    """
    xs = cell_slices(x, L, nsub, t0).astype(np.int64)       # [b, k, t, j]
    S = xs.sum(axis=2).transpose(1, 2, 0)                     # [k, j, b]
    S2 = np.einsum("aktj,bktj->kjab", xs, xs, optimize=True)  # [k, j, a, b]
    return S, S2


def sums_fp64(x: np.ndarray, L: int, nsub: int, t0: int = 0):
    """Eq. 1 sums through FP64 batched matrix products.

    Exact: every product is an integer <= 255^2 and every partial sum is an
    integer below 2^53 as long as L * 255^2 < 2^53 (L < 1.38e11), so no
    rounding ever happens. Returned as int64.
    """
    xs = cell_slices(x, L, nsub, t0).astype(np.float64)      # [b, k, t, j]
    xm = xs.transpose(1, 3, 0, 2)                             # [k, j, b, t]
    S = xm.sum(axis=3)
    S2 = xm @ xm.transpose(0, 1, 3, 2)                        # [k, j, b, b]
    return S.astype(np.int64), S2.astype(np.int64)


def covariance_numerators(S: np.ndarray, S2: np.ndarray, L) -> np.ndarray:
    """N_ab = L * S_ab - S_a * S_b, exact in int64 (L^2 times the covariance).

    ``L`` is a scalar or an array broadcastable to S[..., 0] (samples per
    cell). |N_ab| <= L^2 * 255^2 fits int64 for L < 3.6e7.
    """
    L = np.asarray(L, dtype=np.int64)
    Lb = L[..., None, None] if L.ndim else L
    return Lb * S2 - S[..., :, None] * S[..., None, :]


def correlation(S: np.ndarray, S2: np.ndarray, L):
    """Pearson correlation matrix of each cell in FP64 (Sec. 3.2).

    Returns (r [..., nbeam, nbeam] float64, degenerate [...] bool).
    r_ab = N_ab / sqrt(N_aa * N_bb) with both factors converted to FP64 and
    one division by the square root; r_aa = 1 exactly; rows and columns of a
    zero-variance beam are zero off the diagonal and the cell is degenerate.
    """
    N = covariance_numerators(S, S2, L)
    d = np.diagonal(N, axis1=-2, axis2=-1).astype(np.float64)   # N_aa >= 0
    dead = d <= 0
    denom = np.sqrt(d[..., :, None] * d[..., None, :])
    with np.errstate(divide="ignore", invalid="ignore"):
        r = N.astype(np.float64) / denom
    bad = dead[..., :, None] | dead[..., None, :]
    r = np.where(bad, 0.0, r)
    n = r.shape[-1]
    idx = np.arange(n)
    r[..., idx, idx] = 1.0
    return r, dead.any(axis=-1)


def frobenius2(r: np.ndarray) -> np.ndarray:
    """||C||_F^2 = sum_ab r_ab^2 = n + 2 * sum_{a<b} r_ab^2 (FP64), per cell."""
    n = r.shape[-1]
    iu = np.triu_indices(n, 1)
    off = r[..., iu[0], iu[1]]
    return n + 2.0 * np.sum(off * off, axis=-1)
