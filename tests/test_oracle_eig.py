"""Pins for oracle/eig.py: eigendecomposition and statistic (Sec. 3.3, Eq. 2)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ccm, eig

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_corr(rng, n, L=64):
    x = rng.integers(0, 256, size=(n, L, 1), dtype=np.uint8)
    S, S2 = ccm.sums_int64(x, L, 1)
    return ccm.correlation(S, S2, L)[0][0, 0]


def smith_3x3(A):
    """Trigonometric closed form for the eigenvalues of a symmetric 3x3
    (O. K. Smith, CACM 1961), descending."""
    q = np.trace(A) / 3.0
    p1 = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2 * p1
    p = math.sqrt(p2 / 6.0)
    B = (A - q * np.eye(3)) / p
    rr = min(1.0, max(-1.0, np.linalg.det(B) / 2.0))
    phi = math.acos(rr) / 3.0
    l1 = q + 2 * p * math.cos(phi)
    l3 = q + 2 * p * math.cos(phi + 2 * math.pi / 3)
    return np.array([l1, 3 * q - l1 - l3, l3])


def test_2x2_closed_form():
    for rho in (-0.9, -0.3, 0.0, 0.25, 0.99):
        C = np.array([[1.0, rho], [rho, 1.0]])
        w, V = eig.eig_lapack(C)
        np.testing.assert_allclose(w, [1 + abs(rho), 1 - abs(rho)], atol=1e-15)
        wj, _, _, ok = eig.eig_jacobi(C)
        assert ok
        np.testing.assert_allclose(np.sort(wj)[::-1], [1 + abs(rho), 1 - abs(rho)], atol=1e-15)


def test_3x3_worked_example_against_closed_form():
    with open(os.path.join(GOLD, "worked_3x3.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.uint8)[:, :, None]
    S, S2 = ccm.sums_loops(x, g["L"], 1)
    r, _ = ccm.correlation(S, S2, g["L"])
    C = r[0, 0]
    ref = smith_3x3(C)
    w, V = eig.eig_lapack(C)
    np.testing.assert_allclose(w, ref, atol=1e-14)
    wj, Vj, _, ok = eig.eig_jacobi(C)
    np.testing.assert_allclose(np.sort(wj)[::-1], ref, atol=1e-14)
    s = eig.statistic(w[0], ccm.frobenius2(r)[0, 0])
    assert abs(s - ref[0] ** 2 / (ref ** 2).sum()) < 1e-14
    assert abs(s - 0.79767904) < 5e-9       # value quoted to 8 digits


def test_3x3_random_against_closed_form():
    rng = np.random.default_rng(10)
    for _ in range(20):
        C = _rand_corr(rng, 3, 16)
        np.testing.assert_allclose(eig.eig_lapack(C)[0], smith_3x3(C), atol=1e-13)


@pytest.mark.parametrize("n,rho", [(3, 0.5), (7, -0.1), (19, 0.3), (36, 0.05), (72, 0.9)])
def test_equicorrelation_closed_form(n, rho):
    C = (1 - rho) * np.eye(n) + rho * np.ones((n, n))
    w, V = eig.eig_lapack(C)
    l1 = 1 + (n - 1) * rho
    big = max(abs(l1), abs(1 - rho))
    exp = sorted([l1] + [1 - rho] * (n - 1), key=lambda v: -abs(v))
    np.testing.assert_allclose(w, exp, atol=1e-13 * n)
    s = eig.statistic(w[0], ccm.frobenius2(C[None, None])[0, 0])
    s_ref = big ** 2 / (l1 ** 2 + (n - 1) * (1 - rho) ** 2)
    assert abs(s - s_ref) < 1e-13
    if n == 19 and rho == 0.3:
        assert abs(s - 40.96 / 49.78) < 1e-14     # 0.822820...


def test_diag_plus_rank_one_secular_equation():
    # C = I - diag(u^2) + u u^T: unit diagonal; lambda_1 is the root above
    # max(1 - u_b^2) of 1 = sum u_b^2 / (lambda - 1 + u_b^2) (bisection)
    rng = np.random.default_rng(11)
    for n in (5, 19, 36):
        u = rng.uniform(0.1, 0.8, size=n)
        C = np.eye(n) - np.diag(u * u) + np.outer(u, u)
        lo = max(1 - u * u) + 1e-15
        hi = 1 + (u * u).sum() + 1.0
        f = lambda lam: (u * u / (lam - 1 + u * u)).sum() - 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) > 0:
                lo = mid
            else:
                hi = mid
        w, V = eig.eig_lapack(C)
        assert abs(w[0] - 0.5 * (lo + hi)) < 1e-12
        wj, _, _, _ = eig.eig_jacobi(C)
        assert abs(wj.max() - 0.5 * (lo + hi)) < 1e-12


@pytest.mark.parametrize("n", [2, 7, 19, 36])
def test_jacobi_agrees_with_lapack(n):
    rng = np.random.default_rng(12 + n)
    for _ in range(3):
        C = _rand_corr(rng, n, 4 * n)
        w, V = eig.eig_lapack(C)
        wj, Vj, sweeps, ok = eig.eig_jacobi(C)
        assert ok and sweeps <= 15
        wj_s, Vj_s = eig.order_by_magnitude(wj, Vj)
        np.testing.assert_allclose(wj_s, w, atol=1e-12 * abs(w[0]))
        # residual ||C v - lambda v|| and orthogonality of both routes
        for ww, VV in ((w, V), (wj_s, Vj_s)):
            res = np.linalg.norm(C @ VV - VV * ww[None, :], axis=0).max()
            assert res < 50 * n * 2.2e-16 * abs(w[0])
            assert np.abs(VV.T @ VV - np.eye(n)).max() < 50 * n * 2.2e-16
        assert abs(w.sum() - n) < 1e-12 * n
        assert abs((w * w).sum() - ccm.frobenius2(C[None, None])[0, 0]) < 1e-12 * n


def test_statistic_limits():
    for n in (2, 19, 72):
        I = np.eye(n)
        w, _ = eig.eig_lapack(I)
        assert abs(eig.statistic(w[0], ccm.frobenius2(I[None, None])[0, 0]) - 1.0 / n) < 1e-15
        J = np.ones((n, n))
        w, _ = eig.eig_lapack(J)
        assert abs(eig.statistic(w[0], ccm.frobenius2(J[None, None])[0, 0]) - 1.0) < 1e-13


def test_ordering_by_magnitude_and_sign_convention():
    w = np.array([[0.5, -3.0, 2.0]])
    V = np.eye(3)[None]
    ws, Vs = eig.order_by_magnitude(w, V)
    assert ws.tolist() == [[-3.0, 2.0, 0.5]]
    assert Vs[0][:, 0].tolist() == [0.0, 1.0, 0.0]
    v = eig.fix_sign(np.array([[-0.6, 0.2, 0.1], [0.5, -0.5, 0.0], [0.0, -0.5, 0.5]]))
    assert v[0].tolist() == [0.6, -0.2, -0.1]
    assert v[1].tolist() == [0.5, -0.5, 0.0]
    assert v[2].tolist() == [0.0, 0.5, -0.5]


def test_injected_common_signal_population_eigenvalue():
    """A signal common to all beams with per-beam gain g_b over independent
    noise gives, at large L, the population correlation
    I - diag(u^2) + u u^T with u_b^2 = var(g_b s) / (var(g_b s) + var(noise_b));
    the oracle's sample lambda_1 converges to its secular-equation root."""
    rng = np.random.default_rng(13)
    n, L = 19, 1 << 16
    t = np.arange(L)
    sig = np.rint(10 * np.sin(2 * np.pi * t / 64.0))              # integer, common
    g = rng.uniform(0.5, 1.5, size=n)
    noise = rng.integers(-40, 41, size=(n, L))                    # uniform, var = (81^2-1)/12
    x = np.rint(128 + g[:, None] * sig[None, :]) + noise
    x = x.astype(np.uint8)[:, :, None]
    S, S2 = ccm.sums_int64(x, L, 1)
    r, _ = ccm.correlation(S, S2, L)
    w, _ = eig.eig_lapack(r[0, 0])
    # population quantities from the actual integer signal per beam
    sb = np.rint(128 + g[:, None] * sig[None, :])
    vs = sb.var(axis=1)
    vn = (81 ** 2 - 1) / 12.0
    u = np.sqrt(vs / (vs + vn))
    lo, hi = max(1 - u * u) + 1e-15, 1 + (u * u).sum() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (u * u / (mid - 1 + u * u)).sum() > 1:
            lo = mid
        else:
            hi = mid
    lam_pop = 0.5 * (lo + hi)
    # sampling error of lambda_1 is O(sqrt(n / L)) relative; allow 4 %
    assert abs(w[0] - lam_pop) / lam_pop < 0.04
    assert w[0] > 1 + 0.5 * (n - 1) * (u * u).min()


# ---------------------------------------------------------------------------
# Pins of cell_eigen's dominant eigenvector v1 (Sec. 3.3: the eigenvector of
# the dominant eigenvalue feeds the per-beam stage) against closed forms.

def _unit_with_sign(v):
    """Normalise v and apply the sign convention independently of the oracle:
    sum > 0, or, for a zero sum, the first non-zero component > 0."""
    v = np.asarray(v, dtype=np.float64) / np.linalg.norm(v)
    tot = float(v.sum())
    first = v[np.flatnonzero(v)[0]]
    if tot < 0 or (tot == 0 and first < 0):
        v = -v
    return v


def test_v1_2x2_closed_form():
    # [[1, rho], [rho, 1]]: lambda_1 = 1 + |rho| with v1 = (1, sign rho) / sqrt 2
    rhos = np.array([-0.9, -0.3, 0.25, 0.99])
    C = np.stack([np.array([[1.0, r], [r, 1.0]]) for r in rhos])
    w, v1 = eig.cell_eigen(C)
    for i, r in enumerate(rhos):
        exp = np.array([1.0, math.copysign(1.0, r)]) / math.sqrt(2.0)
        np.testing.assert_allclose(v1[i], exp, atol=1e-15)
        assert abs(w[i, 0] - (1 + abs(r))) < 1e-15


@pytest.mark.parametrize("n,rho", [(3, 0.5), (19, 0.3), (36, 0.05), (72, 0.9)])
def test_v1_equicorrelation_is_uniform(n, rho):
    # (1 - rho) I + rho 11^T, rho > 0: v1 = 1 / sqrt(n) (simple eigenvalue)
    C = (1 - rho) * np.eye(n) + rho * np.ones((n, n))
    _, v1 = eig.cell_eigen(C)
    np.testing.assert_allclose(v1, np.full(n, 1.0 / math.sqrt(n)), atol=1e-13)


def _secular_root(u):
    lo = max(1 - u * u) + 1e-15
    hi = 1 + (u * u).sum() + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (u * u / (mid - 1 + u * u)).sum() > 1:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("n", [4, 19, 36])
def test_v1_diag_plus_rank_one(n):
    """C = I - diag(u^2) + u u^T: (C - lambda I) v = 0 gives
    v_b = u_b (u.v) / (lambda - 1 + u_b^2), so v1 is proportional to
    u_b / (lambda_1 - 1 + u_b^2). Unequal, mixed-sign u makes V non-symmetric
    (a row taken for a column fails) and exercises the sign convention."""
    rng = np.random.default_rng(20 + n)
    for trial in range(4):
        u = rng.uniform(0.1, 0.8, size=n) * np.where(rng.uniform(size=n) < 0.4, -1.0, 1.0)
        if trial == 0:
            u = -np.abs(u)            # sum of v1 negative before the convention
        C = np.eye(n) - np.diag(u * u) + np.outer(u, u)
        lam = _secular_root(u)
        exp = _unit_with_sign(u / (lam - 1 + u * u))
        w, v1 = eig.cell_eigen(C[None])
        assert abs(w[0, 0] - lam) < 1e-12
        np.testing.assert_allclose(v1[0], exp, atol=1e-12)
        assert v1[0].sum() > 0


def test_v1_worked_3x3_against_cross_product():
    """Independent route for a 3x3: v1 spans the null space of C - lambda_1 I,
    i.e. the cross product of two of its rows; lambda_1 from Smith's closed form."""
    with open(os.path.join(GOLD, "worked_3x3.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.uint8)[:, :, None]
    S, S2 = ccm.sums_loops(x, g["L"], 1)
    r, _ = ccm.correlation(S, S2, g["L"])
    C = r[0, 0]
    lam = smith_3x3(C)[0]
    M = C - lam * np.eye(3)
    cands = [np.cross(M[0], M[1]), np.cross(M[0], M[2]), np.cross(M[1], M[2])]
    v = max(cands, key=np.linalg.norm)
    exp = _unit_with_sign(v)
    _, v1 = eig.cell_eigen(C[None])
    np.testing.assert_allclose(v1[0], exp, atol=1e-12)
    np.testing.assert_allclose(C @ v1[0], lam * v1[0], atol=1e-13)


def test_v1_sign_convention_ties():
    # two beams anti-correlated: v1 = (1, -1)/sqrt 2 has a zero sum, so the
    # first non-zero component is made positive
    C = np.array([[[1.0, -0.5], [-0.5, 1.0]]])
    _, v1 = eig.cell_eigen(C)
    np.testing.assert_allclose(v1[0], [1 / math.sqrt(2), -1 / math.sqrt(2)], atol=1e-15)
    # block structure: v1 lives on beams 1, 2 only (beam 0 uncorrelated)
    C = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, -0.8], [0.0, -0.8, 1.0]])
    _, v1 = eig.cell_eigen(C[None])
    np.testing.assert_allclose(v1[0], [0.0, 1 / math.sqrt(2), -1 / math.sqrt(2)], atol=1e-15)
