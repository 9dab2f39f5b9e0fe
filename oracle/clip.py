"""Oracle: iterative Gaussian clipping of the statistic into the RFI mask.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3.3 (paragraph after Fig. 3) and Sec. 4.5 (eigenvalue threshold): after
all cells are processed, the mean and standard deviation of the dominant
eigenvalues are estimated by a Gaussian fit to their distribution, cells whose
value exceeds a dynamic threshold (an integer multiple kappa of the standard
deviation above the mean, kappa = 3 for the FAST data) are masked, and this is
repeated until convergence; the result is a combined mask over channels and
sub-intervals. User-specified frequency ranges can be preserved (Sec. 4.3).

Readings taken where the paper is silent:

* Gaussian fit = moment fit: mean and population standard deviation (ddof 0)
  of the currently unmasked values.
* One-sided, strict: flag s > mu + kappa * sigma.
* Cumulative: a masked cell is never unmasked; stop when an iteration masks
  nothing new, or after ``max_iter`` iterations.
* Scope: one fit over every cell of the block (all channels and sub-ints).
* Eligible cells: not protected and not degenerate; the others are excluded
  from the fit and never masked.
* The clip sees the statistic on a fixed grid of 2^-40: q = rint(s * 2^40),
  s_q = q * 2^-40 (exact in FP64). The moments are exact integer sums
  N, Q1 = sum q, Q2 = sum q^2, so that they do not depend on summation
  order; mu = Q1 / (N 2^40) and var = (N Q2 - Q1^2) / (N^2 2^80) are each
  rounded once to FP64 from the exact rational; sigma = sqrt(var) and
  thr = mu + kappa * sigma in FP64; a cell is masked when s_q > thr. (Using
  s_q rather than s in the comparison keeps a set of equal values, whose
  sigma is 0, unmasked.)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q_SHIFT = 40


def quantize(s: np.ndarray) -> np.ndarray:
    """q = rint(s * 2^40) (FP64 product by a power of two is exact; rint
    rounds half to even). Valid for 0 <= s <= 1."""
    return np.rint(np.asarray(s, dtype=np.float64) * float(1 << Q_SHIFT)).astype(np.int64)


def moments_from_sums(N: int, Q1: int, Q2: int):
    """(mu, sigma) from exact integer moment sums, each rounded once."""
    if N <= 0:
        return math.nan, math.nan
    mu = Q1 / (N << Q_SHIFT)                      # exact rational -> FP64
    var = (N * Q2 - Q1 * Q1) / ((N * N) << (2 * Q_SHIFT))
    return mu, math.sqrt(var)


def dequantize(q: np.ndarray) -> np.ndarray:
    """s_q = q * 2^-40, exact in FP64."""
    return np.asarray(q, dtype=np.int64).astype(np.float64) * 2.0 ** -Q_SHIFT


def exact_sums(q: np.ndarray):
    """(N, sum q, sum q^2) as Python integers."""
    qi = [int(v) for v in np.asarray(q).ravel()]
    return len(qi), sum(qi), sum(v * v for v in qi)


@dataclass
class ClipResult:
    mask: np.ndarray          # bool, same shape as s
    mu: float
    sigma: float
    thr: float
    iterations: int
    converged: bool
    nflag: int


def clip_iterative(s: np.ndarray, eligible: np.ndarray, kappa: float = 3.0,
                   max_iter: int = 50, prior=(0, 0, 0), fit: str = "moments") -> ClipResult:
    """Route 1: the iteration as stated, one pass per iteration.

    ``prior`` = (N_h, Q1_h, Q2_h) are moment sums pooled into every fit (the
    streaming reading of ``clip_stream``); (0, 0, 0) is the paper's batch
    clip. ``fit`` = "histogram" replaces the moment fit by ``fit_histogram``
    of the live values (no prior then).
    """
    eligible = np.asarray(eligible, dtype=bool)
    q = quantize(s)
    sq = dequantize(q)
    masked = np.zeros(sq.shape, dtype=bool)
    Nh, Q1h, Q2h = prior
    mu = sigma = thr = math.nan
    it = 0
    converged = True
    while True:
        live = eligible & ~masked
        N, Q1, Q2 = exact_sums(q[live])
        if N + Nh == 0:
            break
        it += 1
        if fit == "histogram":
            mu, sigma = fit_histogram(sq[live], N, Q1, Q2)
        else:
            mu, sigma = moments_from_sums(N + Nh, Q1 + Q1h, Q2 + Q2h)
        thr = mu + kappa * sigma
        new = live & (sq > thr)
        if not new.any():
            break
        masked |= new
        if it >= max_iter:
            # capped: the last iteration still masked something
            converged = False
            break
    return ClipResult(masked, mu, sigma, thr, it, converged, int(masked.sum()))


def clip_sorted(s: np.ndarray, eligible: np.ndarray, kappa: float = 3.0,
                max_iter: int = 50, prior=(0, 0, 0)) -> ClipResult:
    """Route 2: the same fixed point through sorted prefix sums.

    The masked set is always an upper set {s > T} of the eligible values (the
    running minimum T of the thresholds), so each iteration is a prefix of the
    eligible values sorted ascending; its moment sums come from integer
    prefix sums and the cut from a binary search.
    """
    eligible = np.asarray(eligible, dtype=bool)
    sq = dequantize(quantize(s))
    vals = np.sort(sq[eligible], kind="stable")
    qs = [int(v) for v in quantize(vals)]
    P1 = [0]
    P2 = [0]
    for v in qs:
        P1.append(P1[-1] + v)
        P2.append(P2[-1] + v * v)
    Nh, Q1h, Q2h = prior
    m = len(vals)                 # live cells = vals[:m]
    mu = sigma = thr = math.nan
    it = 0
    converged = True
    T = math.inf
    while m + Nh > 0:
        it += 1
        mu, sigma = moments_from_sums(m + Nh, P1[m] + Q1h, P2[m] + Q2h)
        thr = mu + kappa * sigma
        m_new = int(np.searchsorted(vals[:m], thr, side="right"))
        if m_new == m:
            break
        m = m_new
        T = min(T, thr)
        if it >= max_iter:
            converged = False
            break
    mask = np.zeros(sq.shape, dtype=bool)
    if m < len(vals):
        cut = vals[m]             # smallest masked value
        mask = eligible & (sq >= cut)
    return ClipResult(mask, mu, sigma, thr, it, converged, int(mask.sum()))


HIST_BINS = 64


def histogram_counts(sq_live: np.ndarray, mu_m: float, sig_m: float) -> np.ndarray:
    """Counts of the live values in 64 bins of width sigma_m / 8 over
    [mu_m - 4 sigma_m, mu_m + 4 sigma_m): bin i holds the values with
    floor((v - lo) / w) = i, lo = mu_m - 4 sigma_m, w = sigma_m / 8 (each
    step one FP64 rounding, in this order); values outside are not counted."""
    lo = mu_m - 4.0 * sig_m
    w = sig_m * 0.125
    idx = np.floor((np.asarray(sq_live, dtype=np.float64) - lo) / w)
    counts = np.zeros(HIST_BINS, dtype=np.int64)
    for i in range(HIST_BINS):
        counts[i] = int(np.count_nonzero(idx == i))
    return counts


def fit_histogram(sq_live: np.ndarray, N: int, Q1: int, Q2: int):
    """Gaussian fit to the histogram of the live values (Sec. 3.3, Fig. 1:
    the mean and standard deviation come from a Gaussian fitted to the
    distribution; the paper does not state the bins or the fitting method).

    Reading: the moment fit (mu_m, sigma_m) places 64 bins over +-4 sigma_m
    (``histogram_counts``); ln c_i is fitted by a parabola a + b z + c z^2 in
    the standardised bin centres z_i = (i + 1/2) / 8 - 4 by least squares
    with weights c_i^2 over the non-empty bins (Guo's weighting of Caruana's
    method), solved by Cramer's rule; then mu = mu_m + (-b / 2c) sigma_m and
    sigma = sqrt(-1 / 2c) sigma_m. Fewer than 3 non-empty bins, fewer than 8
    values, sigma_m = 0 or c >= 0 fall back to the moment fit. Sums run over
    the bins in index order, in the operation order written here.
    """
    mu_m, sig_m = moments_from_sums(N, Q1, Q2)
    if N < 8 or not (sig_m > 0):
        return mu_m, sig_m
    counts = histogram_counts(sq_live, mu_m, sig_m)
    if int(np.count_nonzero(counts)) < 3:
        return mu_m, sig_m
    S0 = S1 = S2 = S3 = S4 = T0 = T1 = T2 = 0.0
    for i in range(HIST_BINS):
        c = int(counts[i])
        if c == 0:
            continue
        z = (i + 0.5) * 0.125 - 4.0
        y = math.log(c)
        wt = float(c) * float(c)
        z2 = z * z
        S0 += wt
        S1 += wt * z
        S2 += wt * z2
        S3 += wt * (z2 * z)
        S4 += wt * (z2 * z2)
        T0 += wt * y
        T1 += wt * (z * y)
        T2 += wt * (z2 * y)
    # Cramer's rule for [[S0 S1 S2] [S1 S2 S3] [S2 S3 S4]] (a b c)^T = (T0 T1 T2)^T
    m0 = S2 * S4 - S3 * S3
    m1 = S1 * S4 - S3 * S2
    m2 = S1 * S3 - S2 * S2
    det = S0 * m0 - S1 * m1 + S2 * m2
    if not (det != 0.0):
        return mu_m, sig_m
    db = S0 * (T1 * S4 - S3 * T2) - T0 * m1 + S2 * (S1 * T2 - T1 * S2)
    dc = S0 * (S2 * T2 - T1 * S3) - S1 * (S1 * T2 - T1 * S2) + T0 * m2
    b = db / det
    c2 = dc / det
    if not (c2 < 0.0):
        return mu_m, sig_m
    mu_z = -b / (2.0 * c2)
    sig_z = math.sqrt(-1.0 / (2.0 * c2))
    return mu_m + mu_z * sig_m, sig_z * sig_m


@dataclass
class ScopedResult:
    mask: np.ndarray          # union of the requested scopes' masks [nsub, nchan]
    glob: "ClipResult | None"
    chan: list                # ClipResult per channel (or [])
    sub: list                 # ClipResult per sub-interval (or [])


SCOPE_GLOBAL, SCOPE_CHANNEL, SCOPE_SUBINT = 1, 2, 4


def clip_scoped(s2d: np.ndarray, elig2d: np.ndarray, kappa: float = 3.0, max_iter: int = 50,
                scopes: int = SCOPE_GLOBAL, fit: str = "moments") -> ScopedResult:
    """Clip scopes over the [nsub, nchan] statistic (Sec. 3.3: outliers are
    masked as a function of frequency and time): the global clip over every
    cell, one clip per channel over its sub-intervals, one clip per
    sub-interval over its channels; the result is the union of the masks of
    the requested scopes (the combined mask of Sec. 3.3)."""
    s2d = np.asarray(s2d, dtype=np.float64)
    elig2d = np.asarray(elig2d, dtype=bool)
    nsub, nchan = s2d.shape
    mask = np.zeros((nsub, nchan), dtype=bool)
    g = None
    ch, sb = [], []
    if scopes & SCOPE_GLOBAL:
        g = clip_iterative(s2d.ravel(), elig2d.ravel(), kappa, max_iter, fit=fit)
        mask |= g.mask.reshape(nsub, nchan)
    if scopes & SCOPE_CHANNEL:
        for j in range(nchan):
            r = clip_iterative(s2d[:, j], elig2d[:, j], kappa, max_iter, fit=fit)
            ch.append(r)
            mask[:, j] |= r.mask
    if scopes & SCOPE_SUBINT:
        for k in range(nsub):
            r = clip_iterative(s2d[k, :], elig2d[k, :], kappa, max_iter, fit=fit)
            sb.append(r)
            mask[k, :] |= r.mask
    return ScopedResult(mask, g, ch, sb)


@dataclass
class StreamState:
    """Per-stream pooled history (the serving reading of the clip).

    The paper thresholds once per observation (Sec. 3.3: after the whole
    observation). A stream that delivers an observation block by block keeps
    the exact moment sums of every previously unmasked cell and pools them into
    each later block's fit; with an empty history this is the batch clip.
    """
    N: int = 0
    Q1: int = 0
    Q2: int = 0
    history: list = field(default_factory=list)   # (mu, sigma, thr, iterations)


def clip_stream(state: StreamState, s: np.ndarray, eligible: np.ndarray,
                kappa: float = 3.0, max_iter: int = 50) -> ClipResult:
    """Clip one block against the stream's pooled history, then fold the
    block's final unmasked cells into the history."""
    res = clip_iterative(s, eligible, kappa, max_iter, prior=(state.N, state.Q1, state.Q2))
    live = np.asarray(eligible, dtype=bool) & ~res.mask
    N, Q1, Q2 = exact_sums(quantize(np.asarray(s)[live]))
    state.N += N
    state.Q1 += Q1
    state.Q2 += Q2
    state.history.append((res.mu, res.sigma, res.thr, res.iterations))
    return res
