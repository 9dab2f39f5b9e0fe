"""Pins for oracle/clip.py: iterative Gaussian clipping (Sec. 3.3, Sec. 4.5)."""
import json
import math
import os
import statistics

import numpy as np
import pytest

from oracle import clip

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def naive_clip(s, eligible, kappa, max_iter=50):
    """Brute force on floats: statistics.fmean / pstdev of the unmasked
    values, one pass per iteration (no quantisation, no integer sums)."""
    s = [float(v) for v in s]
    elig = list(eligible)
    masked = [False] * len(s)
    it = 0
    thr = math.nan
    while True:
        vals = [v for v, e, m in zip(s, elig, masked) if e and not m]
        if not vals:
            break
        it += 1
        mu = statistics.fmean(vals)
        sd = statistics.pstdev(vals, mu)
        thr = mu + kappa * sd
        new = [i for i, (v, e, m) in enumerate(zip(s, elig, masked)) if e and not m and v > thr]
        if not new:
            break
        for i in new:
            masked[i] = True
        if it >= max_iter:
            break
    return np.array(masked), it, thr


def test_worked_example():
    with open(os.path.join(GOLD, "worked_clip.json")) as f:
        g = json.load(f)
    s = np.array(g["s"])
    ok = np.ones(s.size, bool)
    for fn in (clip.clip_iterative, clip.clip_sorted):
        res = fn(s, ok, g["kappa"])
        assert sorted(np.nonzero(res.mask)[0].tolist()) == g["mask_indices"]
        assert res.iterations == g["iterations"] and res.converged
        assert abs(res.thr - g["thresholds_6dp"][-1]) < 5e-7
    m, it, thr = naive_clip(s, ok, g["kappa"])
    assert sorted(np.nonzero(m)[0].tolist()) == g["mask_indices"]


def test_exact_moments_match_float_moments():
    rng = np.random.default_rng(20)
    s = rng.uniform(0.05, 1.0, size=5000)
    q = clip.quantize(s)
    N, Q1, Q2 = clip.exact_sums(q)
    mu, sd = clip.moments_from_sums(N, Q1, Q2)
    assert abs(mu - math.fsum(s) / N) < 2e-12
    assert abs(sd - np.std(s)) < 1e-11
    # quantisation: |q 2^-40 - s| <= 2^-41
    assert np.abs(q * 2.0 ** -40 - s).max() <= 2.0 ** -41


def _contaminated(rng, n=3000, frac=0.05):
    s = 0.07 + 0.002 * rng.standard_normal(n)
    k = int(frac * n)
    idx = rng.choice(n, size=k, replace=False)
    s[idx] += rng.uniform(0.005, 0.5, size=k)
    return np.clip(s, 1 / 19, 1.0)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kappa", [2.0, 3.0, 5.0])
def test_two_routes_and_brute_force_agree(seed, kappa):
    rng = np.random.default_rng(100 + seed)
    s = _contaminated(rng)
    ok = rng.uniform(size=s.size) > 0.05
    a = clip.clip_iterative(s, ok, kappa)
    b = clip.clip_sorted(s, ok, kappa)
    assert np.array_equal(a.mask, b.mask)
    assert a.iterations == b.iterations and a.converged == b.converged
    assert a.mu == b.mu and a.sigma == b.sigma and a.thr == b.thr
    m, it, thr = naive_clip(s, ok, kappa)
    assert np.array_equal(a.mask, m) and it == a.iterations
    assert abs(thr - a.thr) < 1e-11


def test_fixed_point_and_upper_set():
    rng = np.random.default_rng(30)
    s = _contaminated(rng, 4000, 0.1)
    ok = np.ones(s.size, bool)
    r = clip.clip_iterative(s, ok, 3.0)
    assert r.converged
    live = ~r.mask
    assert s[live].max() <= r.thr
    assert s[r.mask].min() > s[live].max()          # masked set = {s > cut}
    # the reported fit is the fit of the final unmasked set
    assert abs(r.mu - s[live].mean()) < 1e-12
    assert abs(r.sigma - s[live].std()) < 1e-11


def test_monotone_in_kappa():
    rng = np.random.default_rng(31)
    s = _contaminated(rng, 4000, 0.08)
    ok = np.ones(s.size, bool)
    prev = None
    for kappa in (5.0, 4.0, 3.0, 2.5):
        m = clip.clip_iterative(s, ok, kappa).mask
        if prev is not None:
            assert (m | ~prev).all() and m.sum() >= prev.sum()   # prev subset of m
        prev = m


def test_ineligible_cells_never_masked_and_excluded():
    rng = np.random.default_rng(32)
    s = _contaminated(rng, 2000, 0.05)
    ok = np.ones(s.size, bool)
    big = np.argsort(s)[-20:]
    ok[big[:10]] = False
    r = clip.clip_iterative(s, ok, 3.0)
    assert not r.mask[big[:10]].any()
    r2 = clip.clip_iterative(np.delete(s, big[:10]), np.ones(s.size - 10, bool), 3.0)
    assert r2.thr == r.thr and r2.nflag == r.nflag


def test_max_iter_cap_reports_unconverged():
    # geometric tail: each iteration peels one value
    s = np.concatenate([np.full(50, 0.1), 0.1 + 0.02 * 1.6 ** np.arange(12)])
    ok = np.ones(s.size, bool)
    full = clip.clip_iterative(s, ok, 2.0)
    assert full.converged and full.iterations > 3
    for fn in (clip.clip_iterative, clip.clip_sorted):
        capped = fn(s, ok, 2.0, max_iter=2)
        assert not capped.converged and capped.iterations == 2
    m, it, _ = naive_clip(s, ok, 2.0, max_iter=2)
    assert np.array_equal(m, clip.clip_iterative(s, ok, 2.0, max_iter=2).mask)


def test_degenerate_inputs():
    ok = np.ones(5, bool)
    r = clip.clip_iterative(np.full(5, 0.3), ok, 3.0)
    assert r.nflag == 0 and r.sigma == 0.0 and r.iterations == 1
    r = clip.clip_iterative(np.full(5, 0.3), np.zeros(5, bool), 3.0)
    assert r.nflag == 0 and r.iterations == 0 and math.isnan(r.mu)
    r = clip.clip_iterative(np.array([0.2]), np.ones(1, bool), 3.0)
    assert r.nflag == 0 and r.sigma == 0.0


def test_stream_reduces_to_batch_and_pools_history():
    rng = np.random.default_rng(33)
    s1 = _contaminated(rng, 2000, 0.05)
    s2 = _contaminated(rng, 1500, 0.02)
    ok1, ok2 = np.ones(s1.size, bool), np.ones(s2.size, bool)
    st = clip.StreamState()
    r1 = clip.clip_stream(st, s1, ok1, 3.0)
    b1 = clip.clip_iterative(s1, ok1, 3.0)
    assert np.array_equal(r1.mask, b1.mask) and r1.thr == b1.thr
    live = ~r1.mask
    assert st.N == live.sum()
    assert st.Q1 == sum(int(v) for v in clip.quantize(s1[live]))
    r2 = clip.clip_stream(st, s2, ok2, 3.0)
    # the pooled fit of block 2 is the batch fit over block 2 plus block 1's
    # unmasked cells, with block 1's cells never re-masked
    pooled = np.concatenate([s1[live], s2])
    elig = np.concatenate([np.ones(live.sum(), bool), ok2])
    prior_only = np.zeros(pooled.size, bool)
    prior_only[:live.sum()] = True
    # emulate: iterate on pooled set where prior cells can never be masked
    masked = np.zeros(pooled.size, bool)
    while True:
        v = pooled[~masked]
        thr = v.mean() + 3.0 * v.std()
        new = ~masked & ~prior_only & (pooled > thr)
        if not new.any():
            break
        masked |= new
    assert np.array_equal(masked[live.sum():], r2.mask)
    assert abs(thr - r2.thr) < 1e-11
    assert len(st.history) == 2 and st.N == live.sum() + (~r2.mask).sum()


# ---------------------------------------------------------------------------
# Clip scopes and the histogram Gaussian fit (Sec. 3.3: outliers are masked
# as a function of frequency and time; the mean and standard deviation come
# from a Gaussian fitted to the distribution, Fig. 1).

def _qlive(rng, n, mu=0.075, sd=0.002):
    s = np.clip(mu + sd * rng.standard_normal(n), 0, 1)
    q = clip.quantize(s)
    return clip.dequantize(q), clip.exact_sums(q)


def test_histogram_fit_matches_weighted_polyfit():
    """The Cramer's-rule least squares of fit_histogram against numpy.polyfit
    (weights w_i = c_i multiply the residuals, i.e. c_i^2 weighting) on the
    same bins."""
    rng = np.random.default_rng(61)
    for n in (500, 5000, 60000):
        sq, (N, Q1, Q2) = _qlive(rng, n)
        mu_m, sg_m = clip.moments_from_sums(N, Q1, Q2)
        c = clip.histogram_counts(sq, mu_m, sg_m)
        nz = c > 0
        z = (np.arange(clip.HIST_BINS) + 0.5) * 0.125 - 4.0
        c2, b, a = np.polyfit(z[nz], np.log(c[nz]), 2, w=c[nz].astype(float))
        mu_ref = mu_m + (-b / (2 * c2)) * sg_m
        sd_ref = math.sqrt(-1.0 / (2 * c2)) * sg_m
        mu, sd = clip.fit_histogram(sq, N, Q1, Q2)
        assert abs(mu - mu_ref) <= 1e-12 * mu_ref
        assert abs(sd - sd_ref) <= 1e-9 * sd_ref
        assert c.sum() == np.count_nonzero(np.abs(sq - mu_m) < 4 * sg_m + 1e-18) or c.sum() <= n


def test_histogram_fit_recovers_gaussian_and_symmetry():
    rng = np.random.default_rng(62)
    sq, (N, Q1, Q2) = _qlive(rng, 200000, 0.1, 0.003)
    mu, sd = clip.fit_histogram(sq, N, Q1, Q2)
    assert abs(mu - 0.1) < 5e-5 and abs(sd / 0.003 - 1) < 0.02
    # exactly symmetric values about their mean: the parabola's vertex is the mean
    q = clip.quantize(np.clip(0.2 + 0.004 * rng.standard_normal(4000), 0, 1))
    centre = int(clip.quantize(np.array([0.2]))[0])
    qs = np.concatenate([q, 2 * centre - q])
    N, Q1, Q2 = clip.exact_sums(qs)
    mu_m, _ = clip.moments_from_sums(N, Q1, Q2)
    mu, _ = clip.fit_histogram(clip.dequantize(qs), N, Q1, Q2)
    assert abs(mu - mu_m) <= 1e-12 * mu_m
    # too few values or no spread: the moment fit
    sq, (N, Q1, Q2) = _qlive(rng, 5)
    assert clip.fit_histogram(sq, N, Q1, Q2) == clip.moments_from_sums(N, Q1, Q2)


def test_histogram_clip_flags_outliers():
    rng = np.random.default_rng(63)
    s = np.clip(0.075 + 0.002 * rng.standard_normal(3000), 0, 1)
    bad = rng.choice(3000, 60, replace=False)
    s[bad] += rng.uniform(0.02, 0.5, 60)
    res = clip.clip_iterative(s, np.ones(3000, bool), 3.0, 50, fit="histogram")
    assert res.mask[bad].all() and res.converged
    assert res.mask.sum() < 80


def test_scopes_orientation_and_union():
    """One sub-interval raised in every channel and one channel raised in every
    sub-interval: the per-channel clips catch the raised sub-interval (an
    outlier within each channel) but not the raised channel (uniform within
    it); the per-sub-interval clips the reverse; the union holds both."""
    rng = np.random.default_rng(64)
    K, F = 40, 60
    s = 0.075 + 0.002 * rng.standard_normal((K, F))
    s[7, :] += 0.05                   # broadband burst in sub-interval 7
    s[:, 11] += 0.05                  # persistent RFI in channel 11
    ok = np.ones((K, F), bool)
    ch = clip.clip_scoped(s, ok, scopes=clip.SCOPE_CHANNEL)
    sb = clip.clip_scoped(s, ok, scopes=clip.SCOPE_SUBINT)
    un = clip.clip_scoped(s, ok, scopes=clip.SCOPE_CHANNEL | clip.SCOPE_SUBINT)
    assert ch.mask[7, :].sum() >= F - 1 and ch.mask[:, 11].sum() <= 2
    assert sb.mask[:, 11].sum() >= K - 1 and sb.mask[7, :].sum() <= 2
    assert np.array_equal(un.mask, ch.mask | sb.mask)
    assert len(ch.chan) == F and len(sb.sub) == K
    # per-channel scope == the batch clip of each column on its own
    for j in (0, 11, F - 1):
        r = clip.clip_iterative(s[:, j], ok[:, j])
        assert np.array_equal(ch.mask[:, j], r.mask) and ch.chan[j].thr == r.thr
    g = clip.clip_scoped(s, ok, scopes=clip.SCOPE_GLOBAL)
    assert g.mask[7, :].all() and g.mask[:, 11].all()
