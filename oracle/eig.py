"""Oracle: eigendecomposition of the CCM and the dominant-eigenvalue statistic.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3.3, Eq. 2: C = Q Lambda Q^-1. The eigenvalues are ordered by magnitude,
largest first, and normalised by squaring each and dividing by the sum of all
squared eigenvalues. The statistic used for flagging is the normalised
dominant eigenvalue

    s = lambda_1^2 / sum_i lambda_i^2 = lambda_1^2 / ||C||_F^2

(the two denominators are equal for a symmetric matrix). Its eigenvector q_1
is kept for the per-beam stage (Sec. 3.3, last paragraph); its sign is fixed
here so that sum_b q_1b > 0 (ties: first non-zero component positive).

Two independent routes are provided so that each pins the other:
``eig_lapack`` (numpy.linalg.eigh, LAPACK) and ``eig_jacobi`` (the cyclic-by-row
two-sided Jacobi method of Golub & Van Loan, Matrix Computations, Sec. 8.5,
with the relative skip rule of Demmel & Veselic 1992), both in FP64.
"""
from __future__ import annotations

import math

import numpy as np


def order_by_magnitude(w: np.ndarray, V: np.ndarray | None = None):
    """Sort eigenvalues (last axis) by |lambda| descending (Sec. 3.3)."""
    idx = np.argsort(-np.abs(w), axis=-1, kind="stable")
    w_sorted = np.take_along_axis(w, idx, axis=-1)
    if V is None:
        return w_sorted, None
    V_sorted = np.take_along_axis(V, idx[..., None, :], axis=-1)
    return w_sorted, V_sorted


def fix_sign(v: np.ndarray) -> np.ndarray:
    """Sign convention for an eigenvector (last axis): sum > 0; if the sum is
    exactly 0, the first non-zero component is positive."""
    v = np.array(v, dtype=np.float64, copy=True)
    tot = v.sum(axis=-1)
    nz_first = np.take_along_axis(
        v, np.argmax(v != 0, axis=-1)[..., None], axis=-1)[..., 0]
    flip = (tot < 0) | ((tot == 0) & (nz_first < 0))
    v[flip] = -v[flip]
    return v


def eig_lapack(r: np.ndarray):
    """All eigenpairs of each symmetric matrix by LAPACK (numpy.linalg.eigh),
    ordered by |lambda| descending; eigenvector columns in V[..., :, i]."""
    w, V = np.linalg.eigh(r)
    return order_by_magnitude(w, V)


def eig_jacobi(A: np.ndarray, max_sweeps: int = 50, eps: float = 2.0 ** -52):
    """Cyclic-by-row two-sided Jacobi for one symmetric matrix, FP64.

    Each step zeroes a_pq with the symmetric 2x2 Schur rotation
    (theta = (a_qq - a_pp) / (2 a_pq), t = sign(theta) / (|theta| +
    sqrt(1 + theta^2)), c = 1/sqrt(1+t^2), s = t c) applied as A <- J^T A J
    and V <- V J. A rotation is skipped when |a_pq| <= eps*sqrt(|a_pp a_qq|).
    Sweeps stop after one without rotations. Returns (w, V, sweeps, converged)
    with w unsorted (the final diagonal).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    for sweep in range(1, max_sweeps + 1):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if abs(apq) <= eps * math.sqrt(abs(A[p, p] * A[q, q])):
                    continue
                rotated = True
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(1.0 + theta * theta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                # columns p, q: A <- A J
                Ap = A[:, p].copy()
                Aq = A[:, q].copy()
                A[:, p] = c * Ap - s * Aq
                A[:, q] = s * Ap + c * Aq
                # rows p, q: A <- J^T A
                Ap = A[p, :].copy()
                Aq = A[q, :].copy()
                A[p, :] = c * Ap - s * Aq
                A[q, :] = s * Ap + c * Aq
                A[p, q] = A[q, p] = 0.0
                Vp = V[:, p].copy()
                Vq = V[:, q].copy()
                V[:, p] = c * Vp - s * Vq
                V[:, q] = s * Vp + c * Vq
        if not rotated:
            return np.diag(A).copy(), V, sweep, True
    return np.diag(A).copy(), V, max_sweeps, False


def statistic(lam1, frob2):
    """Normalised dominant eigenvalue s = lambda_1^2 / sum_i lambda_i^2
    (Sec. 3.3), with sum_i lambda_i^2 = ||C||_F^2."""
    lam1 = np.asarray(lam1, dtype=np.float64)
    return lam1 * lam1 / np.asarray(frob2, dtype=np.float64)


def cell_eigen(r: np.ndarray):
    """Per-cell eigen outputs for a stack of correlation matrices.

    Returns (w [..., n] ordered by |lambda| desc, v1 [..., n] unit norm with
    the sign convention of ``fix_sign``).
    """
    w, V = eig_lapack(r)
    v1 = fix_sign(V[..., :, 0])
    return w, v1
