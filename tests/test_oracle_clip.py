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
