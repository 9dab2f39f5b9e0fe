"""Pins for oracle/ccm.py: exact sums and the Pearson CCM (Sec. 3.2, Eq. 1)."""
import json
import os

import numpy as np
import pytest

from oracle import ccm, eig

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_worked_example_sums_and_r():
    g = _load("worked_sums.json")
    x = np.array(g["x"], dtype=np.uint8)[:, :, None]      # [beam, t, chan=1]
    S, S2 = ccm.sums_loops(x, g["L"], 1)
    assert S[0, 0].tolist() == g["S"]
    assert S2[0, 0].tolist() == g["S2"]
    N = ccm.covariance_numerators(S, S2, g["L"])
    assert N[0, 0].tolist() == g["N"]
    r, deg = ccm.correlation(S, S2, g["L"])
    assert not deg[0, 0]
    np.testing.assert_allclose(r[0, 0], np.array(g["r"]), rtol=0, atol=1e-15)


def test_three_routes_agree_bitwise():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(5, 3 * 7, 4), dtype=np.uint8)
    a = ccm.sums_loops(x, 7, 3)
    b = ccm.sums_int64(x, 7, 3)
    c = ccm.sums_fp64(x, 7, 3)
    for u, v in ((a, b), (a, c)):
        assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1])


def test_fp64_route_exact_at_extreme_values():
    # all-255 samples: S_ab = 255^2 L, the largest possible sums
    x = np.full((3, 4 * 4096, 2), 255, dtype=np.uint8)
    S, S2 = ccm.sums_fp64(x, 4096, 4)
    assert (S == 255 * 4096).all() and (S2 == 255 * 255 * 4096).all()


def test_t0_offset_selects_the_right_window():
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, size=(3, 50, 5), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, 8, 4, t0=9)
    S_ref, S2_ref = ccm.sums_loops(x[:, 9:9 + 32, :], 8, 4)
    assert np.array_equal(S, S_ref) and np.array_equal(S2, S2_ref)


def test_correlation_equals_numpy_corrcoef():
    # library special case: Pearson correlation of the float samples
    rng = np.random.default_rng(3)
    x = np.clip(np.rint(128 + 20 * rng.standard_normal((6, 2 * 300, 3))), 0, 255).astype(np.uint8)
    S, S2 = ccm.sums_int64(x, 300, 2)
    r, deg = ccm.correlation(S, S2, 300)
    for k in range(2):
        for j in range(3):
            ref = np.corrcoef(x[:, k * 300:(k + 1) * 300, j].astype(np.float64))
            np.testing.assert_allclose(r[k, j], ref, rtol=0, atol=2e-15)


def test_correlation_properties_and_affine_invariance():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 100, size=(7, 256, 2), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, 256, 1)
    r, _ = ccm.correlation(S, S2, 256)
    c = r[0, 0]
    assert np.array_equal(c, c.T)
    assert (np.diag(c) == 1.0).all() and (np.abs(c) <= 1.0).all()
    assert np.linalg.eigvalsh(c).min() > -1e-12
    # per-beam x -> alpha_b x + beta_b with alpha_b > 0 leaves r unchanged
    alpha = np.array([1, 2, 1, 2, 1, 2, 1])[:, None, None]
    beta = np.array([0, 3, 50, 1, 100, 7, 155])[:, None, None]
    y = (alpha * x.astype(np.int64) + beta).astype(np.uint8)
    Sy, S2y = ccm.sums_int64(y, 256, 1)
    ry, _ = ccm.correlation(Sy, S2y, 256)
    np.testing.assert_allclose(ry, r, rtol=0, atol=1e-14)
    # x -> 255 - x in one beam flips the sign of its row and column
    z = x.copy()
    z[3] = 255 - z[3]
    Sz, S2z = ccm.sums_int64(z, 256, 1)
    rz, _ = ccm.correlation(Sz, S2z, 256)
    sign = np.ones(7)
    sign[3] = -1
    np.testing.assert_allclose(rz[0, 0], c * sign[:, None] * sign[None, :], atol=1e-14)


def test_covariance_numerator_shift_invariant():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 128, size=(4, 64, 1), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, 64, 1)
    y = (x.astype(np.int64) + 100).astype(np.uint8)
    Sy, S2y = ccm.sums_int64(y, 64, 1)
    assert np.array_equal(ccm.covariance_numerators(S, S2, 64),
                          ccm.covariance_numerators(Sy, S2y, 64))


def test_degenerate_beam():
    rng = np.random.default_rng(6)
    x = rng.integers(0, 256, size=(4, 32, 1), dtype=np.uint8)
    x[2] = 77
    S, S2 = ccm.sums_int64(x, 32, 1)
    r, deg = ccm.correlation(S, S2, 32)
    assert deg[0, 0]
    assert r[0, 0, 2, 2] == 1.0
    assert (r[0, 0, 2, [0, 1, 3]] == 0).all() and (r[0, 0, [0, 1, 3], 2] == 0).all()
    # the other beams keep their correlation
    ref = np.corrcoef(x[[0, 1, 3], :, 0].astype(np.float64))
    np.testing.assert_allclose(r[0, 0][np.ix_([0, 1, 3], [0, 1, 3])], ref, atol=1e-14)


def test_frobenius_equals_sum_of_squared_eigenvalues():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, size=(19, 2 * 128, 3), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, 128, 2)
    r, _ = ccm.correlation(S, S2, 128)
    f2 = ccm.frobenius2(r)
    w = np.linalg.eigvalsh(r)
    np.testing.assert_allclose(f2, (w * w).sum(-1), rtol=1e-13)
    np.testing.assert_allclose(f2, (r * r).sum((-1, -2)), rtol=1e-14)
    np.testing.assert_allclose(w.sum(-1), 19.0, rtol=1e-13)


def test_worked_3x3_frobenius():
    g = _load("worked_3x3.json")
    x = np.array(g["x"], dtype=np.uint8)[:, :, None]
    S, S2 = ccm.sums_loops(x, g["L"], 1)
    assert ccm.covariance_numerators(S, S2, g["L"])[0, 0].tolist() == g["N"]
    r, _ = ccm.correlation(S, S2, g["L"])
    assert abs(ccm.frobenius2(r)[0, 0] - g["frob2_num"] / g["frob2_den"]) < 1e-15


# ---------------------------------------------------------------------------
# Long sub-intervals (Table 1 runs sub-intervals of 0.05 - 10 s; 10 s of
# 49.152 us samples is L = 203,450): the sums leave int32 (255^2 L > 2^31 for
# L > 33,025) and the routes must stay exact.

@pytest.mark.parametrize("L", [40960, 203450])
def test_long_cells_exact_against_brute_force(L):
    rng = np.random.default_rng(L)
    nb, nc = 2, 1
    x = rng.integers(0, 256, size=(nb, L, nc), dtype=np.uint8)
    x[0, :34000, 0] = 255                           # saturated: S_aa > 255^2 33025 > 2^31
    # brute force with Python integers, written out independently of sums_loops
    xa = [int(v) for v in x[0, :, 0]]
    xb = [int(v) for v in x[1, :, 0]]
    Sa, Sb = sum(xa), sum(xb)
    Saa = sum(v * v for v in xa)
    Sab = sum(u * v for u, v in zip(xa, xb))
    Sbb = sum(v * v for v in xb)
    for route in (ccm.sums_int64, ccm.sums_fp64):
        S, S2 = route(x, L, 1)
        assert S[0, 0].tolist() == [Sa, Sb]
        assert S2[0, 0].tolist() == [[Saa, Sab], [Sab, Sbb]]
    assert Saa > 2 ** 31                            # beyond the int32 range
    N = ccm.covariance_numerators(S, S2, L)
    assert N[0, 0, 0, 1] == L * Sab - Sa * Sb
    assert N[0, 0, 0, 0] == L * Saa - Sa * Sa


def test_long_cell_all_255_and_alternating():
    # x = 255 everywhere: S_ab = 255^2 L; alternating 0 / 255: the largest
    # variance; the two beams exactly anti-correlated give r = -1
    L = 203450
    x = np.zeros((3, L, 1), dtype=np.uint8)
    x[0] = 255
    x[1, ::2, 0] = 255
    x[2, 1::2, 0] = 255
    S, S2 = ccm.sums_fp64(x, L, 1)
    assert S[0, 0, 0] == 255 * L and S2[0, 0, 0, 0] == 255 * 255 * L
    assert S2[0, 0, 1, 2] == 0 and S2[0, 0, 1, 1] == 255 * 255 * (L // 2)
    r, deg = ccm.correlation(S, S2, L)
    assert deg[0, 0]                                # beam 0 is constant
    assert r[0, 0, 1, 2] == -1.0 and r[0, 0, 0, 1] == 0.0


def test_long_cell_correlation_equals_numpy_corrcoef():
    rng = np.random.default_rng(9)
    L = 81920
    x = np.clip(np.rint(128 + 30 * rng.standard_normal((4, L, 2))), 0, 255).astype(np.uint8)
    x[1] = np.clip(x[0].astype(np.int64) // 2 + x[1] // 2, 0, 255).astype(np.uint8)
    S, S2 = ccm.sums_int64(x, L, 1)
    r, _ = ccm.correlation(S, S2, L)
    for j in range(2):
        ref = np.corrcoef(x[:, :, j].astype(np.float64))
        np.testing.assert_allclose(r[0, j], ref, atol=1e-13)
