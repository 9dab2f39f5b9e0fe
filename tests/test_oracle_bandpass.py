"""Pins for oracle/bandpass.py: ArPLS bandpass (Sec. 3.1, parameters of
Sec. 4.5) and the non-centred CCM of the bandpass-subtracted power."""
import numpy as np
import pytest
import scipy.linalg

from oracle import bandpass, ccm


def test_second_difference_of_a_quadratic():
    F = 12
    j = np.arange(F, dtype=float)
    D = bandpass.second_difference(F)
    np.testing.assert_allclose(D @ (3 * j * j - 5 * j + 7), np.full(F - 2, 6.0), atol=1e-12)
    np.testing.assert_allclose(D @ (4 * j - 1), 0.0, atol=1e-12)


def test_linear_bandpass_is_reproduced_exactly():
    # D y = 0 for a linear y: (W + H) y = W y for every weight vector
    y = 100.0 + 0.25 * np.arange(200)
    z, passes = bandpass.arpls(y, lam=1e6, ratio=0.05, itermax=50)
    np.testing.assert_allclose(z, y, rtol=1e-10)


def test_first_pass_equals_banded_solver():
    """First pass (w = 1): (I + lam D^T D) z = y, against LAPACK's symmetric
    banded solver on the pentadiagonal system."""
    rng = np.random.default_rng(71)
    F, lam = 300, 1e4
    y = 50 + np.cumsum(rng.standard_normal(F))
    z, _ = bandpass.arpls(y, lam=lam, ratio=0.05, itermax=1)
    D = bandpass.second_difference(F)
    A = np.eye(F) + lam * (D.T @ D)
    ab = np.zeros((3, F))                              # upper form, bandwidth 2
    for k in range(3):
        ab[2 - k, k:] = np.diag(A, k)
    zb = scipy.linalg.solveh_banded(ab, y)
    np.testing.assert_allclose(z, zb, rtol=1e-9, atol=1e-9)


def test_asymmetric_reweighting_ignores_positive_rfi():
    """A smooth bandpass plus strong positive narrowband spikes: the reweighted
    fit stays on the bandpass (spikes get weight ~0), while the plain penalised
    fit (one pass, all weights 1) is pulled up towards them."""
    rng = np.random.default_rng(73)
    F = 256
    j = np.arange(F)
    base = 120 + 20 * np.sin(j / 40.0)
    y = base + rng.standard_normal(F)              # the channel means carry noise
    spikes = [30, 31, 90, 150, 151, 152, 200]
    y[spikes] += 80.0
    z1, _ = bandpass.arpls(y, lam=1e4, ratio=1e-6, itermax=1)
    z, passes = bandpass.arpls(y, lam=1e4, ratio=0.05, itermax=100)
    assert passes > 1
    err_plain = np.abs(z1 - base)[spikes].max()
    err = np.abs(z - base)[spikes].max()
    assert err < 0.1 * err_plain and err < 1.0
    assert np.abs(z - base).max() < 1.5


def test_noncentred_ccm_special_cases():
    rng = np.random.default_rng(72)
    L = 512
    x = rng.integers(0, 256, size=(5, L, 3), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, L, 1)
    # baseline 0: the raw second moments S_ab / L
    M0 = bandpass.noncentred_ccm(S, S2, L, np.zeros(S.shape))
    np.testing.assert_allclose(M0, S2 / L, rtol=1e-15)
    # baseline = the exact channel means: the covariance N_ab / L^2
    Mc = bandpass.noncentred_ccm(S, S2, L, S / L)
    N = ccm.covariance_numerators(S, S2, L)
    np.testing.assert_allclose(Mc, N / (L * L), rtol=1e-9, atol=1e-9)
    # against the definition on the samples for an arbitrary baseline
    z = rng.uniform(100, 150, size=S.shape)
    M = bandpass.noncentred_ccm(S, S2, L, z)
    xf = x.astype(np.float64)
    for j in range(3):
        d = xf[:, :, j] - z[0, j][:, None]
        np.testing.assert_allclose(M[0, j], d @ d.T / L, rtol=1e-11)


def test_general_statistic_limits():
    for n in (2, 7, 19):
        s, lam1 = bandpass.statistic_general(np.eye(n)[None] * 3.0)
        assert abs(s[0] - 1.0 / n) < 1e-15
        u = np.linspace(1, 2, n)
        s, lam1 = bandpass.statistic_general(np.outer(u, u)[None])
        assert abs(s[0] - 1.0) < 1e-13 and abs(lam1[0] - u @ u) < 1e-12
